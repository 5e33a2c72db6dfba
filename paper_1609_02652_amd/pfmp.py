"""Python binding of libpfmp (ctypes; argument marshalling only).

Every operation runs in the HIP library; PyTorch provides the device buffers and
the stream.  There is no CPU path: when ``libpfmp.so`` is missing, or no GPU is
visible, constructing a :class:`Lattice` raises.

Buffers: canonical fields are torch tensors on the GPU (complex128 spinors
``[Vh, 4, 3]``, gauge ``[V, 4, 3, 3]``, float64 momenta ``[V, 4, 8]``); internal
fields are flat float64 (or float32) tensors of ``pfmp_field_bytes`` bytes.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libpfmp.so")

F64, F32, F16 = 0, 1, 2
FIELD_SPINOR, FIELD_GAUGE, FIELD_MOMENTA = 0, 1, 2
FORCE_HOP, FORCE_CLOVER, FORCE_F32 = 1, 2, 4
MAX_SHIFTS = 128

ERRORS = {-1: "PFMP_ERR_ARG", -2: "PFMP_ERR_HIP", -3: "PFMP_ERR_NOCONV", -4: "PFMP_ERR_OOM", -5: "PFMP_ERR_STATE"}


class PfmpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERRORS.get(code, code), msg))
        self.code = code


class SolverParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("prec", ctypes.c_int),
                ("delta", ctypes.c_double), ("check_every", ctypes.c_int)]


class SolverStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int), ("true_res", ctypes.c_double),
                ("shift_res", ctypes.c_double * MAX_SHIFTS), ("seconds", ctypes.c_double),
                ("kmults", ctypes.c_longlong)]

    def as_dict(self, nshift=0):
        d = {"iters": self.iters, "reliable_updates": self.reliable_updates, "true_res": self.true_res,
             "seconds": self.seconds, "kmults": self.kmults}
        if nshift:
            d["shift_res"] = [self.shift_res[k] for k in range(nshift)]
        return d


MAX_TERMS = 16
TERM_POLY, TERM_POLYCORR, TERM_RATIO, TERM_HEAVY, TERM_POLYQ = 0, 1, 2, 3, 4
TERM_KINDS = {"poly": TERM_POLY, "polycorr": TERM_POLYCORR, "ratio": TERM_RATIO, "heavy": TERM_HEAVY,
              "polyq": TERM_POLYQ}


class Tuning(ctypes.Structure):
    _fields_ = [("zt", ctypes.c_int), ("stream", ctypes.c_int), ("us_Mhat", ctypes.c_double)]


class Term(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("op", ctypes.c_int), ("op2", ctypes.c_int), ("n", ctypes.c_int),
                ("mu", ctypes.c_double), ("nu", ctypes.c_double), ("steps", ctypes.c_int), ("n1", ctypes.c_int)]


class HmcSpec(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("det_op", ctypes.c_int), ("gauge_steps", ctypes.c_int),
                ("tau", ctypes.c_double), ("lam", ctypes.c_double), ("nterms", ctypes.c_int),
                ("terms", ctypes.POINTER(Term)), ("tol", ctypes.c_double), ("maxiter", ctypes.c_int),
                ("exact_start", ctypes.c_int), ("solver_prec", ctypes.c_int), ("ptnet", ctypes.c_void_p),
                ("batch", ctypes.c_int), ("det_steps", ctypes.c_int)]


class TrajStats(ctypes.Structure):
    _fields_ = [("H0", ctypes.c_double), ("H1", ctypes.c_double), ("dH", ctypes.c_double), ("accept", ctypes.c_int),
                ("nsteps", ctypes.c_int), ("nforce", ctypes.c_int * (MAX_TERMS + 1)), ("kmults", ctypes.c_longlong),
                ("solver_iters", ctypes.c_longlong), ("seconds", ctypes.c_double),
                ("parts0", ctypes.c_double * (MAX_TERMS + 3)), ("parts1", ctypes.c_double * (MAX_TERMS + 3)),
                ("nforce_det", ctypes.c_int)]

    def as_dict(self, nterms):
        return {"H0": self.H0, "H1": self.H1, "dH": self.dH, "accept": bool(self.accept), "nsteps": self.nsteps,
                "nforce": [self.nforce[k] for k in range(nterms + 1)], "kmults": self.kmults,
                "solver_iters": self.solver_iters, "seconds": self.seconds,
                "parts0": [self.parts0[k] for k in range(nterms + 3)],
                "parts1": [self.parts1[k] for k in range(nterms + 3)], "nforce_det": self.nforce_det}


_lib = None


def chebyshev(n, mu, nu):
    """Roots z_1..z_n and a_n of the Chebyshev filter (computed by the library)."""
    L = load()
    r = (ctypes.c_double * (2 * n))()
    nm = (ctypes.c_double * 2)()
    rc = L.pfmp_chebyshev(n, mu, nu, r, nm)
    if rc:
        raise PfmpError(rc, "chebyshev")
    return [complex(r[2 * k], r[2 * k + 1]) for k in range(n)], complex(nm[0], nm[1])


def schedule_build(T_lists, S_lists):
    """Merge per-term (integer tick T, float S) schemes (App. B) in the library."""
    L = load()
    n = len(T_lists)
    lens = (ctypes.c_int * n)(*[len(t) for t in T_lists])
    T = [int(v) for t in T_lists for v in t]
    S = [float(v) for s in S_lists for v in s]
    cap = sum(len(t) for t in T_lists)
    Ta = (ctypes.c_int64 * len(T))(*T)
    Sa = (ctypes.c_double * len(S))(*S)
    To = (ctypes.c_int64 * cap)()
    So = (ctypes.c_double * (cap * n))()
    nout = ctypes.c_int()
    rc = L.pfmp_schedule_build(n, lens, Ta, Sa, cap, To, So, ctypes.byref(nout))
    if rc:
        raise PfmpError(rc, "schedule_build")
    m = nout.value
    return [To[k] for k in range(m)], [[So[j * cap + k] for k in range(m)] for j in range(n)]


def load():
    """Load libpfmp.so (built by ``paper_1609_02652_amd.build``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError("libpfmp.so not built: run `python -m paper_1609_02652_amd.build`")
    L = ctypes.CDLL(LIBPATH)
    vp, i, d, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    sig = {
        "pfmp_create": [vp, i, vp, vp],
        "pfmp_destroy": [vp],
        "pfmp_last_error": [vp],
        "pfmp_field_bytes": [vp, i, i],
        "pfmp_index_maps": [vp, vp, vp, vp],
        "pfmp_set_gauge": [vp, vp],
        "pfmp_get_gauge": [vp, vp],
        "pfmp_set_operator": [vp, i, d, d],
        "pfmp_pack_spinor": [vp, vp, vp, i],
        "pfmp_unpack_spinor": [vp, vp, vp, i],
        "pfmp_pack_momenta": [vp, vp, vp],
        "pfmp_unpack_momenta": [vp, vp, vp],
        "pfmp_apply_hop": [vp, i, i, vp, vp],
        "pfmp_apply_clover": [vp, i, i, i, vp, vp],
        "pfmp_apply_M": [vp, i, i, vp, vp, i],
        "pfmp_apply_MdagM": [vp, i, vp, vp, i],
        "pfmp_apply_MdagM_noalloc": [vp, i, vp, vp, i],
        "pfmp_cg_solve": [vp, i, vp, vp, vp, vp],
        "pfmp_cg_multishift": [vp, i, i, vp, vp, vp, vp, vp],
        "pfmp_dot": [vp, vp, vp, vp],
        "pfmp_axpby": [vp, vp, vp, vp, vp],
        "pfmp_convert_spinor": [vp, vp, i, vp, i],
        "pfmp_logdet_action": [vp, i, vp],
        "pfmp_apply_poly": [vp, i, i, vp, vp, vp, vp, vp, i],
        "pfmp_fermion_force": [vp, i, i, vp, vp, vp, i, vp],
        "pfmp_logdet_force": [vp, i, d, vp],
        "pfmp_gauge_force": [vp, d, vp],
        "pfmp_update_momenta": [vp, d, vp, vp],
        "pfmp_update_gauge": [vp, d, vp],
        "pfmp_gauge_action": [vp, d, vp],
        "pfmp_kinetic": [vp, vp, vp],
        "pfmp_chebyshev": [i, d, d, vp, vp],
        "pfmp_schedule_build": [i, vp, vp, vp, i, vp, vp, vp],
        "pfmp_heatbath": [vp, vp, vp, vp],
        "pfmp_hamiltonian": [vp, vp, vp, vp, vp, vp],
        "pfmp_force_norms": [vp, vp, vp, vp],
        "pfmp_set_half_links": [vp, i],
        "pfmp_set_verbose": [vp, i],
        "pfmp_md_evolve": [vp, vp, vp, vp, vp],
        "pfmp_trajectory": [vp, vp, vp, vp, d, vp, vp],
        "pfmp_set_link_reconstruct": [vp, i],
        "pfmp_set_site_order": [vp, i],
        "pfmp_set_link_streaming": [vp, i],
        "pfmp_autotune": [vp, i, vp],
        "pfmp_set_graphs": [vp, i],
        "pfmp_get_link_reconstruct": [vp, vp],
        "pfmp_apply_MdagM_batch": [vp, i, vp, vp, vp, i],
        "pfmp_set_batch_layout": [vp, i],
        "pfmp_cg_solve_batch": [vp, i, vp, vp, vp, vp, vp],
        "pfmp_ptnet_apply": [vp, vp, vp, vp],
        "pfmp_ptnet_grad": [vp, vp, i, i, vp, vp, vp, vp],
        "pfmp_fcg_solve": [vp, i, vp, vp, vp, vp, vp],
        "pfmp_ptnet_train": [vp, vp, i, i, vp, vp, i, d, vp],
        "pfmp_cg_harvest": [vp, i, vp, vp, d, i, i, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = i
    L.pfmp_last_error.restype = ctypes.c_char_p
    L.pfmp_field_bytes.restype = ll
    _lib = L
    return L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _darr(vals):
    a = (ctypes.c_double * len(vals))(*vals)
    return a


class Lattice:
    """A libpfmp context: one lattice, its gauge field and operator slots."""

    def __init__(self, dims, tbc=-1, device="cuda"):
        import torch
        self.torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("libpfmp needs a GPU (none visible)")
        self.lib = load()
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.Vh = self.V // 2
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        d = (ctypes.c_int * 4)(*self.dims)
        rc = self.lib.pfmp_create(d, int(tbc), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc:
            raise PfmpError(rc, "pfmp_create(%s)" % (self.dims,))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.pfmp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc, what=""):
        if rc:
            raise PfmpError(rc, "%s: %s" % (what, self.lib.pfmp_last_error(self.h).decode()))
        return rc

    # ---------------------------------------------------------------- buffers
    def field(self, kind=FIELD_SPINOR, prec=F64, zero=True):
        nb = self.lib.pfmp_field_bytes(self.h, kind, prec)
        if nb <= 0:
            raise PfmpError(-1, "field_bytes")
        t = self.torch.empty((nb + 7) // 8, dtype=self.torch.float64, device=self.device)
        if zero:
            t.zero_()
        return t

    def to_device(self, a):
        t = self.torch.as_tensor(np.ascontiguousarray(a))
        return t.to(self.device)

    # ---------------------------------------------------------------- fields
    def index_maps(self):
        T = self.torch
        lexeo = T.empty((2, self.Vh), dtype=T.int32, device=self.device)
        nbr = T.empty((2, self.Vh, 8), dtype=T.int32, device=self.device)
        sign = T.empty((2, self.Vh, 8), dtype=T.int8, device=self.device)
        self._chk(self.lib.pfmp_index_maps(self.h, _ptr(lexeo), _ptr(nbr), _ptr(sign)), "index_maps")
        return lexeo, nbr, sign

    def set_gauge(self, U):
        Ud = U if self.torch.is_tensor(U) else self.to_device(np.asarray(U, np.complex128))
        Ud = Ud.contiguous()
        self._chk(self.lib.pfmp_set_gauge(self.h, _ptr(Ud)), "set_gauge")
        self.stream.synchronize()

    def link_reconstruct(self, allow=None):
        """Allow / forbid rebuilding the third link row in the hopping kernels; returns
        whether it is in use (only when the links passed the SU(3) check)."""
        if allow is not None:
            self._chk(self.lib.pfmp_set_link_reconstruct(self.h, int(bool(allow))), "set_link_reconstruct")
        a = ctypes.c_int()
        self._chk(self.lib.pfmp_get_link_reconstruct(self.h, ctypes.byref(a)), "get_link_reconstruct")
        return bool(a.value)

    def site_order(self, zt):
        """Visit order of the operator kernels: 0 memory order, zt > 0 groups of zt z-planes."""
        self._chk(self.lib.pfmp_set_site_order(self.h, int(zt)), "set_site_order")

    def verbose(self, level=1):
        """HMC driver progress lines on stderr (one per phase and per merged fermion step)."""
        self._chk(self.lib.pfmp_set_verbose(self.h, int(level)), "set_verbose")

    def half_links(self, on):
        """FP16-storage solver: FP16 copies of links and clover (True, default) or FP32 ones."""
        self._chk(self.lib.pfmp_set_half_links(self.h, int(bool(on))), "set_half_links")

    def link_streaming(self, on):
        self._chk(self.lib.pfmp_set_link_streaming(self.h, int(bool(on))), "set_link_streaming")

    def graphs(self, on):
        """Replay solver iterations as HIP graphs (default) or launch them one by one."""
        self._chk(self.lib.pfmp_set_graphs(self.h, int(bool(on))), "set_graphs")

    def autotune(self, op):
        """Pick the fastest site visit order and link load mode for Mhat of slot op."""
        t = Tuning()
        self._chk(self.lib.pfmp_autotune(self.h, int(op), ctypes.byref(t)), "autotune")
        return {"zt": t.zt, "stream": t.stream, "us_Mhat": t.us_Mhat}

    def get_gauge(self):
        out = self.torch.empty((self.V, 4, 3, 3), dtype=self.torch.complex128, device=self.device)
        self._chk(self.lib.pfmp_get_gauge(self.h, _ptr(out)), "get_gauge")
        return out

    def set_operator(self, op, kappa, csw):
        self._chk(self.lib.pfmp_set_operator(self.h, int(op), float(kappa), float(csw)), "set_operator")

    def pack_spinor(self, psi, prec=F64, out=None):
        src = psi if self.torch.is_tensor(psi) else self.to_device(np.asarray(psi, np.complex128))
        src = src.contiguous()
        out = self.field(FIELD_SPINOR, prec, zero=False) if out is None else out
        self._chk(self.lib.pfmp_pack_spinor(self.h, _ptr(src), _ptr(out), prec), "pack_spinor")
        return out

    def unpack_spinor(self, f, prec=F64):
        out = self.torch.empty((self.Vh, 4, 3), dtype=self.torch.complex128, device=self.device)
        self._chk(self.lib.pfmp_unpack_spinor(self.h, _ptr(f), _ptr(out), prec), "unpack_spinor")
        return out

    def spinor_numpy(self, f, prec=F64):
        return self.unpack_spinor(f, prec).cpu().numpy()

    def pack_momenta(self, P):
        src = P if self.torch.is_tensor(P) else self.to_device(np.asarray(P, np.float64))
        src = src.contiguous()
        out = self.field(FIELD_MOMENTA, F64, zero=False)
        self._chk(self.lib.pfmp_pack_momenta(self.h, _ptr(src), _ptr(out)), "pack_momenta")
        return out

    def unpack_momenta(self, f):
        out = self.torch.empty((self.V, 4, 8), dtype=self.torch.float64, device=self.device)
        self._chk(self.lib.pfmp_unpack_momenta(self.h, _ptr(f), _ptr(out)), "unpack_momenta")
        return out

    # ---------------------------------------------------------------- operators
    def apply_hop(self, out_parity, x, dagger=False, out=None):
        out = self.field(zero=False) if out is None else out
        self._chk(self.lib.pfmp_apply_hop(self.h, out_parity, int(dagger), _ptr(x), _ptr(out)), "apply_hop")
        return out

    def apply_clover(self, op, parity, inverse, x, out=None):
        out = self.field(zero=False) if out is None else out
        self._chk(self.lib.pfmp_apply_clover(self.h, op, parity, int(inverse), _ptr(x), _ptr(out)), "apply_clover")
        return out

    def apply_M(self, op, x, dagger=False, prec=F64, out=None):
        # F16: FP32 fields in and out (FP16 storage inside the library)
        out = self.field(FIELD_SPINOR, F32 if prec == F16 else prec, zero=False) if out is None else out
        self._chk(self.lib.pfmp_apply_M(self.h, op, int(dagger), _ptr(x), _ptr(out), prec), "apply_M")
        return out

    def apply_MdagM(self, op, x, prec=F64, out=None):
        out = self.field(FIELD_SPINOR, F32 if prec == F16 else prec, zero=False) if out is None else out
        self._chk(self.lib.pfmp_apply_MdagM(self.h, op, _ptr(x), _ptr(out), prec), "apply_MdagM")
        return out

    def apply_MdagM_noalloc(self, op, x, out, prec=F64):
        """Khat through the allocation-free entry point (the caller passes out)."""
        self._chk(self.lib.pfmp_apply_MdagM_noalloc(self.h, op, _ptr(x), _ptr(out), prec), "apply_MdagM_noalloc")
        return out

    # ---------------------------------------------------------------- solvers
    @staticmethod
    def params(tol=1e-10, maxiter=10000, prec=F64, delta=0.0, check_every=0):
        return SolverParams(tol, maxiter, prec, delta, check_every)

    def cg_solve(self, op, b, x=None, tol=1e-10, maxiter=10000, prec=F64, delta=0.0, check_every=0, check=True):
        x = self.field(zero=False) if x is None else x
        st = SolverStats()
        p = self.params(tol, maxiter, prec, delta, check_every)
        rc = self.lib.pfmp_cg_solve(self.h, op, _ptr(b), _ptr(x), ctypes.byref(p), ctypes.byref(st))
        if check:
            self._chk(rc, "cg_solve")
        return x, st.as_dict()

    def cg_multishift(self, op, shifts, b, xs=None, tol=1e-10, maxiter=10000, check_every=0):
        z = [float(v) for s in shifts for v in (complex(s).real, complex(s).imag)]
        n = len(shifts)
        xs = [self.field(zero=False) for _ in range(n)] if xs is None else xs
        xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        st = SolverStats()
        p = self.params(tol, maxiter, F64, 0.0, check_every)
        self._chk(self.lib.pfmp_cg_multishift(self.h, op, n, _darr(z), _ptr(b), xp, ctypes.byref(p),
                                              ctypes.byref(st)), "cg_multishift")
        return xs, st.as_dict(n)

    def apply_MdagM_batch(self, ops, xs, outs=None, prec=F64):
        n = len(xs)
        outs = [self.field(prec=prec, zero=False) for _ in range(n)] if outs is None else outs
        o = (ctypes.c_int * n)(*ops)
        ip = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        op_ = (ctypes.c_void_p * n)(*[x.data_ptr() for x in outs])
        self._chk(self.lib.pfmp_apply_MdagM_batch(self.h, n, o, ip, op_, prec), "apply_MdagM_batch")
        return outs

    def batch_layout(self, multi):
        """Batched clover stencils: True / 1 the default group of rhs per lane pair, 2 or 4
        that many rhs per lane pair, False / 0 one workgroup per (site block, rhs)."""
        self._chk(self.lib.pfmp_set_batch_layout(self.h, int(multi)), "set_batch_layout")

    def cg_solve_batch(self, ops, bs, xs=None, tol=1e-10, maxiter=10000, check_every=0, prec=F64):
        n = len(bs)
        xs = [self.field(zero=False) for _ in range(n)] if xs is None else xs
        o = (ctypes.c_int * n)(*ops)
        bp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in bs])
        xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        st = (SolverStats * n)()
        p = self.params(tol, maxiter, prec, 0.0, check_every)
        self._chk(self.lib.pfmp_cg_solve_batch(self.h, n, o, bp, xp, ctypes.byref(p), st), "cg_solve_batch")
        return xs, [st[k].as_dict() for k in range(n)]

    # ---------------------------------------------------------------- learned preconditioner
    @staticmethod
    def _weights(W):
        """(W1, W2, W0) complex arrays -> 1568 doubles [W1 | W2 | W0]."""
        flat = np.concatenate([np.asarray(w, np.complex128).ravel() for w in W])
        assert flat.size == 784
        return np.ascontiguousarray(flat.view(np.float64))

    @staticmethod
    def _unweights(a):
        c = np.asarray(a, np.float64).view(np.complex128)
        return c[:384].reshape(8, 12, 4), c[384:768].reshape(8, 4, 12), c[768:].reshape(4, 4)

    def ptnet_apply(self, W, r, out=None):
        out = self.field(zero=False) if out is None else out
        w = self._weights(W)
        self._chk(self.lib.pfmp_ptnet_apply(self.h, w.ctypes.data_as(ctypes.c_void_p), _ptr(r), _ptr(out)),
                  "ptnet_apply")
        return out

    @staticmethod
    def _training_set(data, op):
        """(r pointers, e pointers or None) of a training set: vectors r (op given, the
        preconditioned-residual objective) or pairs (r, e) with Khat e = r."""
        if op is None:
            rs, es = [p[0] for p in data], [p[1] for p in data]
        else:
            rs, es = [p[0] if isinstance(p, (tuple, list)) else p for p in data], None
        n = len(rs)
        rp = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rs])
        ep = (ctypes.c_void_p * n)(*[e.data_ptr() for e in es]) if es is not None else None
        return n, rp, ep

    def ptnet_grad(self, W, data, op=None):
        """Loss and gradient matrices (A1, A2, A0) of the training objective: with op, the
        preconditioned residual sum |Khat_op z(rhat) - rhat|^2 over vectors r; without,
        solution matching over pairs (r, e)."""
        n, rp, ep = self._training_set(data, op)
        w = self._weights(W)
        loss = ctypes.c_double()
        A = np.zeros(1568)
        self._chk(self.lib.pfmp_ptnet_grad(self.h, w.ctypes.data_as(ctypes.c_void_p), -1 if op is None else int(op),
                                           n, rp, ep, ctypes.byref(loss), A.ctypes.data_as(ctypes.c_void_p)),
                  "ptnet_grad")
        return loss.value, self._unweights(A)

    def ptnet_train(self, W, data, steps, lr=1e-2, op=None):
        """Adam in the library; returns the trained (W1, W2, W0) and the loss history."""
        n, rp, ep = self._training_set(data, op)
        w = self._weights(W).copy()
        losses = np.zeros(steps)
        self._chk(self.lib.pfmp_ptnet_train(self.h, w.ctypes.data_as(ctypes.c_void_p), -1 if op is None else int(op),
                                            n, rp, ep, int(steps), float(lr),
                                            losses.ctypes.data_as(ctypes.c_void_p)), "ptnet_train")
        return self._unweights(w), losses

    def fcg_solve(self, op, W, b, x=None, tol=1e-10, maxiter=10000, check=True):
        x = self.field(zero=False) if x is None else x
        st = SolverStats()
        p = self.params(tol, maxiter)
        wp = None
        if W is not None:
            w = self._weights(W)
            wp = w.ctypes.data_as(ctypes.c_void_p)
        rc = self.lib.pfmp_fcg_solve(self.h, op, wp, _ptr(b), _ptr(x), ctypes.byref(p), ctypes.byref(st))
        if check:
            self._chk(rc, "fcg_solve")
        return x, st.as_dict()

    def cg_harvest(self, op, b, snap_iters, tol=1e-10, maxiter=10000):
        """Solve Khat x = b and return (x, [(r_k, e_k = x - x_k)]) at the given iterations."""
        n = len(snap_iters)
        xs = [self.field(zero=False) for _ in range(n)]
        rs = [self.field(zero=False) for _ in range(n)]
        x = self.field(zero=False)
        it = (ctypes.c_int * max(1, n))(*snap_iters)
        xp = (ctypes.c_void_p * max(1, n))(*[v.data_ptr() for v in xs])
        rp = (ctypes.c_void_p * max(1, n))(*[v.data_ptr() for v in rs])
        taken = ctypes.c_int()
        self._chk(self.lib.pfmp_cg_harvest(self.h, op, _ptr(b), _ptr(x), float(tol), int(maxiter), n, it, xp, rp,
                                           ctypes.byref(taken)), "cg_harvest")
        pairs = []
        for k in range(taken.value):
            e = x.clone()
            self.axpby(-1.0, xs[k], 1.0, e)
            pairs.append((rs[k], e))
        return x, pairs

    # ---------------------------------------------------------------- BLAS
    def dot(self, a, b):
        out = (ctypes.c_double * 2)()
        self._chk(self.lib.pfmp_dot(self.h, _ptr(a), _ptr(b), out), "dot")
        return complex(out[0], out[1])

    def axpby(self, alpha, x, beta, y):
        a = _darr([complex(alpha).real, complex(alpha).imag])
        b = _darr([complex(beta).real, complex(beta).imag])
        self._chk(self.lib.pfmp_axpby(self.h, a, _ptr(x), b, _ptr(y)), "axpby")
        return y

    def convert_spinor(self, x, prec_in, prec_out, out=None):
        out = self.field(FIELD_SPINOR, prec_out, zero=False) if out is None else out
        self._chk(self.lib.pfmp_convert_spinor(self.h, _ptr(x), prec_in, _ptr(out), prec_out), "convert_spinor")
        return out

    # ---------------------------------------------------------------- polynomial
    def apply_poly(self, op, roots, norm, x, out=None, chain=None, prec=F64):
        n = len(roots)
        r = _darr([v for z in roots for v in (complex(z).real, complex(z).imag)]) if n else None
        nm = _darr([complex(norm).real, complex(norm).imag])
        out = self.field(FIELD_SPINOR, prec, zero=False) if out is None else out
        ch = None
        if chain is not None:
            ch = (ctypes.c_void_p * n)(*[c.data_ptr() for c in chain])
        self._chk(self.lib.pfmp_apply_poly(self.h, op, n, r, nm, _ptr(x), _ptr(out), ch, prec), "apply_poly")
        return out

    # ---------------------------------------------------------------- forces and updates
    def fermion_force(self, op, pairs, F, flags=0):
        """F += sum_p d/dw Re[c_p X_p^dag Mhat Y_p] for pairs (X_p, Y_p, c_p)."""
        n = len(pairs)
        xs = (ctypes.c_void_p * n)(*[p[0].data_ptr() for p in pairs])
        ys = (ctypes.c_void_p * n)(*[p[1].data_ptr() for p in pairs])
        cs = _darr([v for p in pairs for v in (complex(p[2]).real, complex(p[2]).imag)])
        self._chk(self.lib.pfmp_fermion_force(self.h, op, n, xs, ys, cs, flags, _ptr(F)), "fermion_force")
        return F

    def logdet_force(self, op, F, coef=1.0):
        self._chk(self.lib.pfmp_logdet_force(self.h, op, float(coef), _ptr(F)), "logdet_force")
        return F

    def gauge_force(self, beta, F):
        self._chk(self.lib.pfmp_gauge_force(self.h, float(beta), _ptr(F)), "gauge_force")
        return F

    def update_momenta(self, eps, F, P):
        self._chk(self.lib.pfmp_update_momenta(self.h, float(eps), _ptr(F), _ptr(P)), "update_momenta")
        return P

    def update_gauge(self, eps, P):
        self._chk(self.lib.pfmp_update_gauge(self.h, float(eps), _ptr(P)), "update_gauge")

    def gauge_action(self, beta):
        out = ctypes.c_double()
        self._chk(self.lib.pfmp_gauge_action(self.h, float(beta), ctypes.byref(out)), "gauge_action")
        return out.value

    def kinetic(self, P):
        out = ctypes.c_double()
        self._chk(self.lib.pfmp_kinetic(self.h, _ptr(P), ctypes.byref(out)), "kinetic")
        return out.value

    # ---------------------------------------------------------------- HMC
    @staticmethod
    def spec(beta, terms, gauge_steps, det_op=-1, tau=1.0, lam=0.0, tol=1e-10, maxiter=100000,
             exact_start=False, solver_prec=F64, ptnet=None, batch=False, det_steps=0):
        """terms: list of dicts {kind, op, op2, n, n1, mu, nu, steps} (kind poly, polycorr, ratio,
        heavy or polyq; n1: the inner degree of polyq); ptnet: (W1, W2, W0) or None; batch: the
        solves of all ratio / heavy terms due at one merged step run as one multi-RHS solve;
        det_steps: S_det on its own 2MN scale (0: with the gauge action)."""
        arr = (Term * max(1, len(terms)))()
        for k, t in enumerate(terms):
            arr[k] = Term(TERM_KINDS[t["kind"]], t["op"], t.get("op2", -1), t.get("n", 0), t.get("mu", 0.0),
                          t.get("nu", 0.0), t["steps"], t.get("n1", 0))
        wp, keep_w = None, None
        if ptnet is not None:
            keep_w = Lattice._weights(ptnet).copy()
            wp = keep_w.ctypes.data
        sp = HmcSpec(beta, det_op, gauge_steps, tau, lam, len(terms), arr, tol, maxiter, int(exact_start),
                     int(solver_prec), wp, int(batch), int(det_steps))
        sp._keep = (arr, keep_w)
        return sp

    def heatbath(self, spec, etas, phis=None):
        n = spec.nterms
        phis = [self.field(zero=False) for _ in range(n)] if phis is None else phis
        e = (ctypes.c_void_p * max(1, n))(*[x.data_ptr() for x in etas])
        p = (ctypes.c_void_p * max(1, n))(*[x.data_ptr() for x in phis])
        self._chk(self.lib.pfmp_heatbath(self.h, ctypes.byref(spec), e, p), "heatbath")
        return phis

    def hamiltonian(self, spec, P, phis):
        n = spec.nterms
        p = (ctypes.c_void_p * max(1, n))(*[x.data_ptr() for x in phis])
        H = ctypes.c_double()
        parts = (ctypes.c_double * (n + 3))()
        self._chk(self.lib.pfmp_hamiltonian(self.h, ctypes.byref(spec), _ptr(P), p, ctypes.byref(H), parts),
                  "hamiltonian")
        return H.value, list(parts)

    def force_norms(self, spec, phis):
        """Rows (gauge, each term, S_det) of (max, mean) over links of |F| at the current links."""
        n = spec.nterms
        p = (ctypes.c_void_p * max(1, n))(*[x.data_ptr() for x in phis])
        out = (ctypes.c_double * (2 * (n + 2)))()
        self._chk(self.lib.pfmp_force_norms(self.h, ctypes.byref(spec), p, out), "force_norms")
        return np.array(list(out)).reshape(n + 2, 2)

    def md_evolve(self, spec, P, phis):
        n = spec.nterms
        p = (ctypes.c_void_p * max(1, n))(*[x.data_ptr() for x in phis])
        st = TrajStats()
        self._chk(self.lib.pfmp_md_evolve(self.h, ctypes.byref(spec), _ptr(P), p, ctypes.byref(st)), "md_evolve")
        return st.as_dict(n)

    def trajectory(self, spec, P0, etas, u, P_end=None):
        n = spec.nterms
        e = (ctypes.c_void_p * max(1, n))(*[x.data_ptr() for x in etas])
        st = TrajStats()
        pe = _ptr(P_end) if P_end is not None else None
        self._chk(self.lib.pfmp_trajectory(self.h, ctypes.byref(spec), _ptr(P0), e, float(u), pe, ctypes.byref(st)),
                  "trajectory")
        return st.as_dict(n)

    def logdet_action(self, op):
        out = ctypes.c_double()
        self._chk(self.lib.pfmp_logdet_action(self.h, op, ctypes.byref(out)), "logdet_action")
        return out.value
