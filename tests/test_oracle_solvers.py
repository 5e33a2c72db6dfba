"""Pins for the oracle's solvers and the Chebyshev polynomial filter (CPU only).

Checks against: dense linear algebra on 4^4, the closed Chebyshev form of
z P_n(z), the normalisation mu P(mu) = 1, the factorisation rule of App. A, the
partial-fraction identity of App. C, and free-field eigenvectors.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import chebyshev
from paper_1609_02652_amd import synth

DIMS = (4, 4, 4, 4)
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def op():
    U = synth.random_gauge(DIMS, seed=0)
    return oracle.Operator(DIMS, U, 0.12, 1.0)


@pytest.fixture(scope="module")
def Kdense(op):
    n = 12 * 128
    K = np.zeros((n, n), np.complex128)
    for j in range(n):
        e = np.zeros((128, 4, 3), np.complex128)
        e.reshape(-1)[j] = 1
        K[:, j] = op.K(e).reshape(-1)
    return K


def test_cg_matches_dense_solve(op, Kdense):
    b = synth.gaussian_spinor(128, 11)
    x, st = op.cg(b, tol=1e-12)
    assert st["rc"] == 0 and st["true_res"] <= 1.05e-12
    xd = np.linalg.solve(Kdense, b.reshape(-1))
    cond = np.linalg.cond(Kdense)
    assert np.linalg.norm(x.reshape(-1) - xd) / np.linalg.norm(xd) <= 2 * cond * 1e-12
    assert np.allclose(Kdense, Kdense.conj().T, atol=1e-13)


def test_cg_reports_nonconvergence(op):
    b = synth.gaussian_spinor(128, 11)
    x, st = op.cg(b, tol=1e-12, maxiter=3)
    assert st["rc"] == -3 and st["iters"] == 3 and st["true_res"] > 1e-6


def test_shifted_solve(op, Kdense):
    b = synth.gaussian_spinor(128, 12)
    z = chebyshev.roots(4, 1.2, 0.9)[1]
    x, st = op.cg_shift(z, b, tol=1e-11)
    assert st["rc"] == 0 and st["true_res"] <= 1e-11
    xd = np.linalg.solve(Kdense - z * np.eye(Kdense.shape[0]), b.reshape(-1))
    assert np.linalg.norm(x.reshape(-1) - xd) / np.linalg.norm(xd) < 1e-9


# ---------------------------------------------------------------- Chebyshev scalars

def cheb_T(k, x):
    """Chebyshev T_k(x) by the three-term recurrence (complex x)."""
    t0, t1 = 1.0 + 0j, x
    if k == 0:
        return t0
    for _ in range(k - 1):
        t0, t1 = t1, 2 * x * t1 - t0
    return t1


@pytest.mark.parametrize("n", [2, 3, 4, 5, 10, 16, 31, 32, 64])
def test_chebyshev_closed_form(n):
    """z P_n(z) is the Chebyshev residual on foci mu +/- nu, derived from the root
    parametrisation of App. A (with mu/nu = cosh e, (mu - z_k)/nu = cosh(e + i th_k),
    so T_{n+1} takes the same value at every root):
        z P_n(z) = [T_{n+1}((mu-z)/nu) - T_{n+1}(mu/nu)] / [T_{n+1}(0) - T_{n+1}(mu/nu)],
    i.e. 1 - T_{n+1}((mu-z)/nu)/T_{n+1}(mu/nu) for even n, where T_{n+1}(0) = 0."""
    mu, nu = 1.2, 0.9
    rng = np.random.default_rng(n)
    for z in list(rng.uniform(0.01, 2.3, 5)) + [0.5 + 0.3j, 1.7 - 0.2j]:
        lhs = z * chebyshev.evaluate(z, n, mu, nu)
        t0, tm = cheb_T(n + 1, 0.0), cheb_T(n + 1, mu / nu)
        rhs = (cheb_T(n + 1, (mu - z) / nu) - tm) / (t0 - tm)
        if n % 2 == 0:
            assert abs(rhs - (1 - cheb_T(n + 1, (mu - z) / nu) / tm)) < 1e-14
        assert abs(lhs - rhs) < 2e-14 * max(1.0, abs(rhs))
    assert abs(mu * chebyshev.evaluate(mu, n, mu, nu) - 1) < 1e-14
    # real polynomial: roots closed under conjugation, a_n real; positive for even n,
    # negative for odd n (the real root 2 mu contributes the factor mu - 2 mu < 0)
    a = chebyshev.norm(n, mu, nu)
    assert abs(a.imag) < 1e-14 * abs(a) and (a.real > 0) == (n % 2 == 0)
    chebyshev.conjugate_partner(chebyshev.roots(n, mu, nu))


@pytest.mark.parametrize("n", [4, 16])
def test_chebyshev_error_bound(n):
    """max over [mu-nu, mu+nu] of |1 - z P(z)| is 1/T_{n+1}(mu/nu) (even n)."""
    mu, nu = 1.2, 0.9
    zs = np.linspace(mu - nu, mu + nu, 4001)
    err = max(abs(1 - z * chebyshev.evaluate(z, n, mu, nu)) for z in zs)
    bound = 1 / cheb_T(n + 1, mu / nu).real
    assert abs(err - bound) < 1e-12 + 1e-9 * bound


def test_factorisation_rule():
    g = json.load(open(os.path.join(GOLD, "chebyshev_params.json")))
    mu, nu = g["mu"], g["nu"]
    for p1, p2 in g["nested_pairs_factorising"]:
        assert (p2 + 1) % (p1 + 1) == 0
        assert chebyshev.divides(p1, p2, mu, nu)
    for p1, p2 in g["pairs_not_factorising"]:
        assert not chebyshev.divides(p1, p2, mu, nu)


def test_quotient_filter():
    """Q = P_p2 / P_p1 (eq. 2poly): Q(z) P_p1(z) = P_p2(z) at points off the roots, p2 - p1
    roots closed under conjugation, a positive norm; the pairs the paper's schemes use
    (p1 = 4 inside p2 = 24 for 2PF-1MP) and the golden factorising pairs."""
    g = json.load(open(os.path.join(GOLD, "chebyshev_params.json")))
    mu, nu = g["mu"], g["nu"]
    rng = np.random.default_rng(7)
    pairs = [(4, 24), (2, 8)] + [tuple(p) for p in g["nested_pairs_factorising"]]
    for p1, p2 in pairs:
        zq, aq = chebyshev.quotient(p2, p1, mu, nu)
        assert len(zq) == p2 - p1
        chebyshev.conjugate_partner(zq)
        assert abs(aq.imag) < 1e-12 * abs(aq) and aq.real > 0
        assert sum(1 for z in zq if z.imag < 0) == (p2 - p1) // 2
        for w in rng.normal(size=6) * 1.5 + 1j * rng.normal(size=6) + 1.0:
            q = aq
            for z in zq:
                q *= (w - z)
            lhs = q * chebyshev.evaluate(w, p1, mu, nu)
            rhs = chebyshev.evaluate(w, p2, mu, nu)
            assert abs(lhs - rhs) < 1e-11 * abs(rhs), (p1, p2, w)
    for p1, p2 in g["pairs_not_factorising"]:
        with pytest.raises(ValueError):
            chebyshev.quotient(p2, p1, mu, nu)


@pytest.mark.parametrize("n", [4, 16, 64])
def test_partial_fractions(n):
    """prod_i 1/(z - z_i) = sum_i r_i / (z - z_i) over the n roots plus z_{n+1} = 0."""
    zs = chebyshev.roots(n, 1.2, 0.9) + [0j]
    r = chebyshev.residues(zs)
    for z in (0.37 + 0.11j, 2.9, -0.4 + 1j):
        prod = 1.0
        for zi in zs:
            prod /= (z - zi)
        terms = [ri / (z - zi) for ri, zi in zip(r, zs)]
        s = sum(terms)
        # rounding bound of the sum: cancellation among large residues
        assert abs(prod - s) < 1e-11 * abs(prod) + 1e-14 * sum(abs(t) for t in terms)


# ---------------------------------------------------------------- operator polynomial

def test_poly_on_free_field_eigenvector():
    """P(K) v = P(lambda) v for a free-field eigenvector of K."""
    U = synth.unit_gauge(DIMS)
    kappa = 0.12
    fop = oracle.Operator(DIMS, U, kappa, 1.0)
    lexeo, _, _ = oracle.index_maps(DIMS)
    n = (1, 0, 2, 1)
    p = [2 * math.pi * n[m] / 4 for m in range(3)] + [2 * math.pi * (n[3] + 0.5) / 4]
    a = 2 * sum(math.cos(q) for q in p)
    b = [2 * math.sin(q) for q in p]
    bn = math.sqrt(sum(x * x for x in b))
    bg = sum(b[m] * oracle.gamma(m) for m in range(4))
    w, vec = np.linalg.eigh(bg)
    u = np.outer(vec[:, int(np.argmin(np.abs(w - bn)))], [1.0, -0.5j, 0.25])
    psi = np.zeros((128, 4, 3), np.complex128)
    for i, x in enumerate(lexeo[0]):
        c = [x % 4, (x // 4) % 4, (x // 16) % 4, x // 64]
        psi[i] = np.exp(1j * sum(p[m] * c[m] for m in range(4))) * u
    lam = abs(1 - kappa ** 2 * (a - 1j * bn) ** 2) ** 2
    assert np.max(np.abs(fop.K(psi) - lam * psi)) < 1e-12
    for deg in (4, 16):
        z = chebyshev.roots(deg, 1.2, 0.9)
        an = chebyshev.norm(deg, 1.2, 0.9)
        got = fop.poly(z, an, psi)
        want = chebyshev.evaluate(lam, deg, 1.2, 0.9) * psi
        assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


def test_pole_sum_equals_product_operator(op):
    """[K P(K)]^-1 phi = (1/a_n) sum_i r_i (K - z_i)^-1 phi (App. C with the 1/a_n of
    the normalisation), checked by CG on the product operator vs shifted solves."""
    n = 4
    z = chebyshev.roots(n, 1.2, 0.9)
    a = chebyshev.norm(n, 1.2, 0.9).real
    zs = z + [0j]
    r = chebyshev.residues(zs)
    phi = synth.gaussian_spinor(128, 21)
    x_prod, st = op.cg_poly(zs, a, phi, tol=1e-12)
    assert st["rc"] == 0 and st["true_res"] < 1.05e-12
    acc = np.zeros_like(phi)
    for ri, zi in zip(r, zs):
        if zi == 0:
            xi, _ = op.cg(phi, tol=1e-13)
        else:
            xi, _ = op.cg_shift(zi, phi, tol=1e-13)
        acc += ri * xi
    acc /= a
    assert np.linalg.norm(acc - x_prod) / np.linalg.norm(x_prod) < 1e-10
