"""PF-MP HMC on the oracle: actions, pseudofermion heatbath, forces, trajectory.

TEST INFRASTRUCTURE ONLY (part of the oracle).

Action (paper eq. pfmp_action, with the even-odd reduction of the clover operator):
  S = S_G + S_det + sum of filter terms,
  S_G   = beta sum_P (1 - Re tr U_P / 3)                        (Wilson gauge action)
  S_det = -2 sum_{x odd} ln det A(x)                             (det M = det A_oo det Mhat)
  'poly'     phi^dag P(J) phi,          P = a_n prod (J - z_k)     (App. A)
  'polyq'    phi^dag Q(J) phi,          Q = P_n / P_n1, the intermediate filter of the
                                       2-filter actions (eq. 2poly; App. A factorisation)
  'polycorr' phi^dag [J P(J)]^-1 phi                              (eq. 1poly, 2nd term)
  'ratio'    phi^dag W_a^dag J_b^-1 W_a phi                        (Hasenbusch ratio J_a J_b^-1,
                                                                   read as W_a^dag J_b^-1 W_a)
  'heavy'    phi^dag J^-1 phi                                     (eq. hasenbusch, 1st term)
with J = W^dag W, W = Mhat at a heavier kappa (K = M^dag M at the target kappa).

Forces are d/dw S along U -> exp(i w T_a) U (coefficients of T_a).  The
polynomial force follows eq. force_poly (vectors chi_i, eta_i built incrementally);
the correction force is computed here WITHOUT the pole sum of eq. force_polycorr:
the oracle differentiates phi^dag B^-1 phi for the product operator
B = J P(J) = a_n prod_{k=1..n+1} (J - z_k), z_{n+1} = 0, with B^-1 phi by CG on B
(the route the paper sets aside for speed), so that it checks the pole sum rather
than repeating it.  Each bilinear derivative comes from Operator.force_bilinear.
"""
import math

import numpy as np

from . import Operator, force_gauge, gauge_action, kinetic, update_gauge, update_momenta
from . import chebyshev, schedule


def _vdot(a, b):
    return np.vdot(a.ravel(), b.ravel())


class Ops:
    """Operators at every kappa an action uses, on one gauge field."""

    def __init__(self, dims, U, csw, tbc=-1):
        self.dims, self.U, self.csw, self.tbc = dims, U, csw, tbc
        self._ops = {}

    def __call__(self, kappa):
        k = float(kappa)
        if k not in self._ops:
            self._ops[k] = Operator(self.dims, self.U, k, self.csw, self.tbc)
        return self._ops[k]


def _J(op, v):
    return op.K(v)


def _prod_vectors(op, roots, a, phi):
    """chi_i = a prod_{j>i} (J - z_j) phi and eta_i = prod_{j<i} (J - z_j^*) phi."""
    n = len(roots)
    chi = [None] * n
    chi[n - 1] = a * phi
    for i in range(n - 1, 0, -1):
        chi[i - 1] = _J(op, chi[i]) - roots[i] * chi[i]
    eta = [None] * n
    eta[0] = phi.copy()
    for i in range(1, n):
        eta[i] = _J(op, eta[i - 1]) - np.conj(roots[i - 1]) * eta[i - 1]
    return chi, eta


def _dJ_pairs(op, X, Y, c=1.0):
    """Re[c X^dag dJ Y] as M-bilinears: Re[c (W X)^dag dW Y] + Re[conj(c) (W Y)^dag dW X]."""
    return [(op.M(X), Y, c), (op.M(Y), X, np.conj(c))]


def term_roots(term):
    if term["kind"] == "polyq":
        z, a = chebyshev.quotient(term["n"], term["n1"], term["mu"], term["nu"])
        return z, a.real
    return chebyshev.roots(term["n"], term["mu"], term["nu"]), chebyshev.norm(term["n"], term["mu"], term["nu"]).real


def heatbath(ops, term, eta):
    """phi with density exp(-S_term) from Gaussian eta (exp(-eta^dag eta))."""
    kind = term["kind"]
    if kind in ("poly", "polyq"):
        # P = R^dag R with R = sqrt(a) prod (J - z_k) over the roots below the real axis
        # (one of each conjugate pair); phi = R^-1 eta.
        op = ops(term["kappa"])
        z, a = term_roots(term)
        half = [r for r in z if r.imag < 0]
        if 2 * len(half) != len(z):
            raise ValueError("heatbath for a polynomial term needs conjugate root pairs (even degree)")
        v = eta / math.sqrt(a)
        for r in half:
            v, st = op.cg_shift(r, v, tol=term.get("tol_hb", 1e-13))
        return v
    if kind == "polycorr":
        # phi = R^dag W^dag eta, R^dag = sqrt(a_n) prod_{k <= n/2} (J - z_k^*)
        op = ops(term["kappa"])
        z, a = term_roots(term)
        n = len(z)
        v = op.M(eta, dagger=True)
        for k in range(n // 2):
            v = _J(op, v) - np.conj(z[k]) * v
        return math.sqrt(a) * v
    if kind == "ratio":
        # phi = J_a^-1 W_a^dag M_b^dag eta
        oa, ob = ops(term["kappa_num"]), ops(term["kappa_den"])
        v = oa.M(ob.M(eta, dagger=True), dagger=True)
        x, st = oa.cg(v, tol=term.get("tol_hb", 1e-13))
        return x
    if kind == "heavy":
        return ops(term["kappa"]).M(eta, dagger=True)
    raise ValueError(kind)


def action(ops, term, phi, tol):
    kind = term["kind"]
    if kind in ("poly", "polyq"):
        op = ops(term["kappa"])
        z, a = term_roots(term)
        return _vdot(phi, op.poly(z, a, phi)).real
    if kind == "polycorr":
        op = ops(term["kappa"])
        z, a = term_roots(term)
        x, st = op.cg_poly(list(z) + [0.0], a, phi, tol=tol)
        return _vdot(phi, x).real
    if kind == "ratio":
        oa, ob = ops(term["kappa_num"]), ops(term["kappa_den"])
        v = oa.M(phi)
        x, st = ob.cg(v, tol=tol)
        return _vdot(v, x).real
    if kind == "heavy":
        op = ops(term["kappa"])
        x, st = op.cg(phi, tol=tol)
        return _vdot(phi, x).real
    raise ValueError(kind)


def force(ops, term, phi, tol, F=None, links=None):
    """F += d S_term / dw (coefficients per link)."""
    V = int(np.prod(ops.dims))
    if F is None:
        F = np.zeros((V, 4, 8))
    kind = term["kind"]
    if kind in ("poly", "polyq"):
        op = ops(term["kappa"])
        z, a = term_roots(term)
        chi, eta = _prod_vectors(op, z, a, phi)
        pairs = []
        for c, e in zip(chi, eta):
            pairs += _dJ_pairs(op, e, c)
        return op.force_bilinear(pairs, F, links)
    if kind == "polycorr":
        # S = phi^dag B^-1 phi, dS = -psi^dag dB psi with psi = B^-1 phi,
        # B = a_n prod_{k=1..n+1} (J - z_k), z_{n+1} = 0.
        op = ops(term["kappa"])
        z, a = term_roots(term)
        zz = list(z) + [0.0]
        psi, st = op.cg_poly(zz, a, phi, tol=tol)
        chi, eta = _prod_vectors(op, zz, a, psi)
        pairs = []
        for c, e in zip(chi, eta):
            pairs += _dJ_pairs(op, e, c, -1.0)
        return op.force_bilinear(pairs, F, links)
    if kind == "ratio":
        # S = v^dag K_b^-1 v with v = W_a phi; X = K_b^-1 v:
        # dS = 2 Re[X^dag dW_a phi] - 2 Re[(M_b X)^dag dM_b X]
        oa, ob = ops(term["kappa_num"]), ops(term["kappa_den"])
        x, st = ob.cg(oa.M(phi), tol=tol)
        oa.force_bilinear([(x, phi, 2.0)], F, links)
        return ob.force_bilinear([(ob.M(x), x, -2.0)], F, links)
    if kind == "heavy":
        op = ops(term["kappa"])
        x, st = op.cg(phi, tol=tol)
        return op.force_bilinear([(op.M(x), x, -2.0)], F, links)
    raise ValueError(kind)


def build_schedule(spec):
    """Per-term 2MN schemes merged per App. B.  Rows: gauge, the terms, and, when
    spec["det_steps"] > 0, S_det on its own scale as the last row (otherwise S_det
    moves with the gauge action on the finest scale)."""
    tau = spec.get("tau", 1)
    lam = spec.get("lambda", schedule.OMELYAN_LAMBDA)
    steps = [spec["gauge_steps"]] + [t["steps"] for t in spec["terms"]]
    if spec.get("det_steps", 0) > 0:
        steps.append(spec["det_steps"])
    Ts, Ss = [], []
    for n in steps:
        T, S = schedule.omelyan_2mn(n, tau, lam)
        Ts.append(T)
        Ss.append(S)
    return schedule.merge(Ts, Ss)


def hamiltonian(spec, U, P, phis, tol):
    dims = spec["dims"]
    ops = Ops(dims, U, spec["csw"], spec.get("tbc", -1))
    parts = {"kinetic": kinetic(P), "gauge": gauge_action(dims, U, spec["beta"]),
             "logdet": ops(spec["kappa"]).logdet_action() if spec["csw"] != 0 else 0.0}
    for i, (t, phi) in enumerate(zip(spec["terms"], phis)):
        parts["term%d" % i] = action(ops, t, phi, tol)
    return sum(parts.values()), parts


def md_evolve(spec, U, P, phis, tol):
    """Molecular dynamics over the merged schedule: for each merged step k, T[dt_k]
    then S_j[eps_jk] for every term with a nonzero step (App. B, enacted loop).
    U and P are updated in place; returns the number of force evaluations per term."""
    dims = spec["dims"]
    newT, newS = build_schedule(spec)
    nforce = [0] * len(newS)
    det_row = len(spec["terms"]) + 1 if spec.get("det_steps", 0) > 0 else 0
    for k, dt in enumerate(newT):
        if dt != 0:
            update_gauge(dims, float(dt), P, U)
        ops = Ops(dims, U, spec["csw"], spec.get("tbc", -1))
        for j, S in enumerate(newS):
            eps = float(S[k])
            if eps == 0:
                continue
            nforce[j] += 1
            if j == 0:
                F = force_gauge(dims, U, spec["beta"])
                if spec["csw"] != 0 and det_row == 0:
                    ops(spec["kappa"]).force_logdet(F)
            elif j == det_row:
                F = np.zeros_like(P)
                if spec["csw"] != 0:
                    ops(spec["kappa"]).force_logdet(F)
            else:
                F = force(ops, spec["terms"][j - 1], phis[j - 1], tol)
            update_momenta(eps, F, P)
    return nforce


def trajectory(spec, U0, P0, etas, u=None, tol=1e-12):
    """One PF-MP HMC trajectory.  Returns the final fields, dH, the accept
    decision for the uniform u, and bookkeeping."""
    dims = spec["dims"]
    U = np.array(U0, dtype=np.complex128, copy=True)
    P = np.array(P0, dtype=np.float64, copy=True)
    ops0 = Ops(dims, U, spec["csw"], spec.get("tbc", -1))
    phis = [heatbath(ops0, t, eta) for t, eta in zip(spec["terms"], etas)]
    H0, parts0 = hamiltonian(spec, U, P, phis, tol)
    nforce = md_evolve(spec, U, P, phis, tol)
    H1, parts1 = hamiltonian(spec, U, P, phis, tol)
    dH = H1 - H0
    out = {"U": U, "P": P, "dH": dH, "H0": H0, "H1": H1, "parts0": parts0, "parts1": parts1,
           "phis": phis, "nforce": nforce}
    if u is not None:
        out["accept"] = bool(u < math.exp(-dH)) if dH > 0 else True
    return out
