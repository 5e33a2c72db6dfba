"""Plain FP64 CPU oracle for the PF-MP HMC hot path (arXiv:1609.02652).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py``; never by the product package.  It shares no code
with the HIP path.  The heavy lattice operators are plain C (``pfmp_oracle.c``);
the host-side scalars (Chebyshev roots, pole residues), the integrator schedule and
the HMC driver are plain Python in ``chebyshev.py``, ``schedule.py`` and ``hmc.py``.

Canonical layouts (numpy, complex128 unless stated):
  gauge   U[V, 4, 3, 3]       lexicographic sites, x fastest
  spinor  psi[Vh, 4, 3]       one parity, even-odd index = lex // 2
  forces  F[V, 4, 8] float64  coefficients of T_a = lambda_a / 2
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "pfmp_oracle.c")


def build(force=True):
    """Compile the C oracle with gcc (plain -O2, OpenMP for timing only)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", _SO, _SRC, "-lm"]
        subprocess.check_call(cmd)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        vp, dp, ip = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p
        L.or_op_create.restype = vp
        L.or_op_create.argtypes = [ip, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double]
        L.or_op_free.argtypes = [vp]
        L.or_index_maps.argtypes = [ip, ctypes.c_int, ip, ip, ip]
        L.or_gamma.argtypes = [ctypes.c_int, dp]
        L.or_generator.argtypes = [ctypes.c_int, dp]
        L.or_clover_at.argtypes = [vp, ctypes.c_long, dp, dp, dp]
        L.or_hop_full.argtypes = [vp, ctypes.c_int, dp, dp]
        L.or_hop_eo.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, dp]
        L.or_apply_clover.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp, dp]
        L.or_apply_M.argtypes = [vp, ctypes.c_int, dp, dp]
        L.or_apply_K.argtypes = [vp, dp, dp]
        L.or_cg.argtypes = [vp, dp, dp, ctypes.c_double, ctypes.c_int, ip, dp]
        L.or_cg.restype = ctypes.c_int
        L.or_cg_shift.argtypes = [vp, ctypes.c_double, ctypes.c_double, dp, dp, ctypes.c_double, ctypes.c_int, ip, dp]
        L.or_cg_shift.restype = ctypes.c_int
        L.or_apply_poly.argtypes = [vp, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.or_cg_poly.argtypes = [vp, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, dp, dp,
                                 ctypes.c_double, ctypes.c_int, ip, dp]
        L.or_cg_poly.restype = ctypes.c_int
        L.or_gauge_action.argtypes = [ip, dp, ctypes.c_double]
        L.or_gauge_action.restype = ctypes.c_double
        L.or_plaquette.argtypes = [ip, dp]
        L.or_plaquette.restype = ctypes.c_double
        L.or_logdet_action.argtypes = [vp]
        L.or_logdet_action.restype = ctypes.c_double
        L.or_force_bilinear.argtypes = [vp, ctypes.c_int, ip, ip, dp, dp, ctypes.c_long, ip]
        L.or_force_logdet.argtypes = [vp, ctypes.c_double, dp, ctypes.c_long, ip]
        L.or_force_gauge.argtypes = [ip, dp, ctypes.c_double, dp, ctypes.c_long, ip]
        L.or_update_gauge.argtypes = [ip, ctypes.c_double, dp, dp]
        L.or_update_momenta.argtypes = [ctypes.c_long, ctypes.c_double, dp, dp]
        L.or_kinetic.argtypes = [ctypes.c_long, dp]
        L.or_kinetic.restype = ctypes.c_double
        L.or_sample_sites.argtypes = [ip, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_int, dp, ctypes.c_long, ip, dp]
        L.or_sample_sites.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(dims):
    return np.ascontiguousarray(dims, dtype=np.int32)


def gamma(mu):
    """Dirac matrix gamma_mu (mu = 0..3), or gamma_5 for mu = 4."""
    out = np.zeros((4, 4), np.complex128)
    lib().or_gamma(mu, _p(out))
    return out


def generator(a):
    """SU(3) generator T_a = lambda_{a+1} / 2, a = 0..7."""
    out = np.zeros((3, 3), np.complex128)
    lib().or_generator(a, _p(out))
    return out


def index_maps(dims, tbc=-1):
    """Brute-force even-odd tables: lex_of_eo[2, Vh], nbr[2, Vh, 8], sign[2, Vh, 8]."""
    d = _dims(dims)
    V = int(np.prod(dims))
    lexeo = np.zeros((2, V // 2), np.int32)
    nbr = np.zeros((2, V // 2, 8), np.int32)
    sign = np.zeros((2, V // 2, 8), np.int8)
    lib().or_index_maps(_p(d), tbc, _p(lexeo), _p(nbr), _p(sign))
    return lexeo, nbr, sign


class Operator:
    """Even-odd Wilson-clover operator at one (kappa, csw) on a gauge field."""

    def __init__(self, dims, U, kappa, csw, tbc=-1):
        self.dims = _dims(dims)
        self.U = np.ascontiguousarray(U, dtype=np.complex128)
        self.V = int(np.prod(dims))
        self.Vh = self.V // 2
        self.kappa, self.csw, self.tbc = float(kappa), float(csw), int(tbc)
        assert self.U.shape == (self.V, 4, 3, 3)
        self.h = lib().or_op_create(_p(self.dims), self.tbc, _p(self.U), self.kappa, self.csw)
        if not self.h:
            raise ValueError("oracle: lattice extents must be even and >= 4")

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_op_free(self.h)
            self.h = None

    def _new(self):
        return np.zeros((self.Vh, 4, 3), np.complex128)

    def hop_eo(self, out_parity, psi, adjoint=False):
        out = self._new()
        lib().or_hop_eo(self.h, out_parity, int(adjoint), _p(np.ascontiguousarray(psi)), _p(out))
        return out

    def hop_full(self, psi, adjoint=False):
        out = np.zeros((self.V, 4, 3), np.complex128)
        lib().or_hop_full(self.h, int(adjoint), _p(np.ascontiguousarray(psi)), _p(out))
        return out

    def clover(self, parity, psi, inverse=False):
        out = self._new()
        lib().or_apply_clover(self.h, parity, int(inverse), _p(np.ascontiguousarray(psi)), _p(out))
        return out

    def clover_at(self, lex):
        A = np.zeros((12, 12), np.complex128)
        Ai = np.zeros((12, 12), np.complex128)
        ld = np.zeros(1, np.complex128)
        lib().or_clover_at(self.h, lex, _p(A), _p(Ai), _p(ld))
        return A, Ai, ld[0]

    def M(self, psi, dagger=False):
        out = self._new()
        lib().or_apply_M(self.h, int(dagger), _p(np.ascontiguousarray(psi)), _p(out))
        return out

    def K(self, psi):
        out = self._new()
        lib().or_apply_K(self.h, _p(np.ascontiguousarray(psi)), _p(out))
        return out

    def cg(self, b, tol=1e-12, maxiter=100000):
        x = self._new()
        it = np.zeros(1, np.int32)
        res = np.zeros(1)
        rc = lib().or_cg(self.h, _p(np.ascontiguousarray(b)), _p(x), tol, maxiter, _p(it), _p(res))
        return x, {"rc": rc, "iters": int(it[0]), "true_res": float(res[0])}

    def cg_shift(self, z, b, tol=1e-12, maxiter=100000):
        """x = (K - z)^-1 b by CG on the normal equations."""
        x = self._new()
        it = np.zeros(1, np.int32)
        res = np.zeros(1)
        rc = lib().or_cg_shift(self.h, float(np.real(z)), float(np.imag(z)), _p(np.ascontiguousarray(b)), _p(x),
                               tol, maxiter, _p(it), _p(res))
        return x, {"rc": rc, "iters": int(it[0]), "true_res": float(res[0])}

    def poly(self, roots, norm, psi):
        """norm * prod_k (K - z_k) psi, factors applied in the order given."""
        r = np.ascontiguousarray(np.asarray(roots, np.complex128))
        out = self._new()
        lib().or_apply_poly(self.h, len(r), _p(r), float(np.real(norm)), float(np.imag(norm)),
                            _p(np.ascontiguousarray(psi)), _p(out))
        return out

    def cg_poly(self, roots, norm, b, tol=1e-12, maxiter=100000):
        """x = [norm * prod_k (K - z_k)]^-1 b by CG on the product operator."""
        r = np.ascontiguousarray(np.asarray(roots, np.complex128))
        x = self._new()
        it = np.zeros(1, np.int32)
        res = np.zeros(1)
        rc = lib().or_cg_poly(self.h, len(r), _p(r), float(np.real(norm)), float(np.imag(norm)),
                              _p(np.ascontiguousarray(b)), _p(x), tol, maxiter, _p(it), _p(res))
        return x, {"rc": rc, "iters": int(it[0]), "true_res": float(res[0])}

    def logdet_action(self):
        return lib().or_logdet_action(self.h)

    def force_bilinear(self, pairs, F=None, links=None):
        """F += sum_p d/dw Re[c_p X_p^dag Mhat Y_p] for pairs (X_p, Y_p, c_p), for every
        link (or only the listed links x*4+mu)."""
        if F is None:
            F = np.zeros((self.V, 4, 8))
        Xs = [np.ascontiguousarray(p[0], dtype=np.complex128) for p in pairs]
        Ys = [np.ascontiguousarray(p[1], dtype=np.complex128) for p in pairs]
        coef = np.ascontiguousarray([[np.real(p[2]), np.imag(p[2])] for p in pairs], dtype=np.float64)
        xp = (ctypes.c_void_p * len(pairs))(*[a.ctypes.data for a in Xs])
        yp = (ctypes.c_void_p * len(pairs))(*[a.ctypes.data for a in Ys])
        ln, lp = _links(links)
        lib().or_force_bilinear(self.h, len(pairs), ctypes.cast(xp, ctypes.c_void_p), ctypes.cast(yp, ctypes.c_void_p),
                                _p(coef), _p(F), ln, lp)
        return F

    def force_logdet(self, F=None, coef=1.0, links=None):
        """F += coef * d/dw S_det, S_det = -2 sum_odd ln det A."""
        if F is None:
            F = np.zeros((self.V, 4, 8))
        ln, lp = _links(links)
        lib().or_force_logdet(self.h, coef, _p(F), ln, lp)
        return F


_keep = []


def _links(links):
    if links is None:
        return 0, None
    arr = np.ascontiguousarray(links, dtype=np.int64)
    _keep.append(arr)
    if len(_keep) > 8:
        del _keep[0]
    return len(arr), _p(arr)


def sample_sites(dims, U, kappa, csw, psi, sites, mode, dagger=False, tbc=-1):
    """The hop D_oe psi (mode "hop": odd output sites) or Mhat psi (mode "M": even
    output sites, dagger for Mhat^dag) at the given even-odd output indices only,
    from the definitions with the clover of the few sites involved built on the
    spot (eq. 2.2; clover and Schur form as in the operator context).  psi: even
    field [Vh][4][3].  Returns [n][4][3]."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    idx = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.zeros((len(idx), 4, 3), np.complex128)
    rc = lib().or_sample_sites(_p(_dims(dims)), tbc, _p(U), kappa, csw, {"hop": 0, "M": 1}[mode], int(dagger),
                               _p(psi), len(idx), _p(idx), _p(out))
    if rc:
        raise ValueError("or_sample_sites failed (%d)" % rc)
    return out


def gauge_action(dims, U, beta):
    return lib().or_gauge_action(_p(_dims(dims)), _p(np.ascontiguousarray(U)), float(beta))


def plaquette(dims, U):
    return lib().or_plaquette(_p(_dims(dims)), _p(np.ascontiguousarray(U)))


def force_gauge(dims, U, beta, F=None, links=None):
    V = int(np.prod(dims))
    if F is None:
        F = np.zeros((V, 4, 8))
    ln, lp = _links(links)
    lib().or_force_gauge(_p(_dims(dims)), _p(np.ascontiguousarray(U)), float(beta), _p(F), ln, lp)
    return F


def update_gauge(dims, eps, P, U):
    """In place: U <- exp(i eps P) U."""
    assert U.flags["C_CONTIGUOUS"] and P.flags["C_CONTIGUOUS"]
    lib().or_update_gauge(_p(_dims(dims)), float(eps), _p(P), _p(U))
    return U


def update_momenta(eps, F, P):
    """In place: P <- P - eps F."""
    lib().or_update_momenta(P.shape[0] * P.shape[1], float(eps), _p(np.ascontiguousarray(F)), _p(P))
    return P


def kinetic(P):
    """sum over links of tr P^2."""
    P = np.ascontiguousarray(P)
    return lib().or_kinetic(P.shape[0] * P.shape[1], _p(P))
