"""Pins for the oracle's forces, integrator and HMC (CPU only).

Forces are checked against central finite differences of the actions they
differentiate; the schedule against the worked example of App. B; the link update
against an independent matrix exponential; the trajectory against reversibility,
dH ~ h^2, the heatbath identity S_i(start) = eta_i^dag eta_i and <exp(-dH)> = 1.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from oracle import hmc, schedule
from paper_1609_02652_amd import synth

DIMS = (4, 4, 4, 4)
V, VH = 256, 128
GOLD = os.path.join(os.path.dirname(__file__), "golden")
T = [oracle.generator(a) for a in range(8)]


def perturbed(U, link, a, w):
    U2 = U.copy()
    x, mu = divmod(link, 4)
    U2[x, mu] = sl.expm(1j * w * T[a]) @ U2[x, mu]
    return U2


def fd(fun, U, link, a, eps=1e-5):
    return (fun(perturbed(U, link, a, eps)) - fun(perturbed(U, link, a, -eps))) / (2 * eps)


SAMPLES = [(0, 0), (37, 3), (101, 7), (530, 5), (1023, 1)]


@pytest.fixture(scope="module")
def U0():
    return synth.random_gauge(DIMS, seed=0)


def test_bilinear_force_fd(U0):
    X = synth.gaussian_spinor(VH, 1)
    Y = synth.gaussian_spinor(VH, 2)
    c = 0.7 - 0.4j
    F = oracle.Operator(DIMS, U0, 0.12, 1.3).force_bilinear([(X, Y, c)])
    fun = lambda U: (c * np.vdot(X, oracle.Operator(DIMS, U, 0.12, 1.3).M(Y))).real
    for link, a in SAMPLES:
        ref = fd(fun, U0, link, a)
        assert abs(F[link // 4, link % 4, a] - ref) < 1e-7 * max(1, abs(ref))


def test_bilinear_force_wilson_fd(U0):
    """c_sw = 0: the paper's even-odd Wilson operator."""
    X = synth.gaussian_spinor(VH, 3)
    Y = synth.gaussian_spinor(VH, 4)
    F = oracle.Operator(DIMS, U0, 0.15, 0.0).force_bilinear([(X, Y, 1.0)])
    fun = lambda U: np.vdot(X, oracle.Operator(DIMS, U, 0.15, 0.0).M(Y)).real
    for link, a in SAMPLES:
        ref = fd(fun, U0, link, a)
        assert abs(F[link // 4, link % 4, a] - ref) < 1e-7 * max(1, abs(ref))


def test_logdet_and_gauge_force_fd(U0):
    F = oracle.Operator(DIMS, U0, 0.13, 1.6).force_logdet()
    G = oracle.force_gauge(DIMS, U0, 5.6)
    fl = lambda U: oracle.Operator(DIMS, U, 0.13, 1.6).logdet_action()
    fg = lambda U: oracle.gauge_action(DIMS, U, 5.6)
    for link, a in SAMPLES:
        assert abs(F[link // 4, link % 4, a] - fd(fl, U0, link, a)) < 1e-7
        assert abs(G[link // 4, link % 4, a] - fd(fg, U0, link, a)) < 1e-6


TERMS = [
    dict(kind="poly", kappa=0.110, n=4, mu=1.2, nu=0.9),
    dict(kind="polycorr", kappa=0.110, n=4, mu=1.2, nu=0.9),
    dict(kind="ratio", kappa_num=0.110, kappa_den=0.120),
    dict(kind="heavy", kappa=0.110),
    dict(kind="polyq", kappa=0.110, n=8, n1=2, mu=1.2, nu=0.9),
]


@pytest.mark.parametrize("term", TERMS, ids=[t["kind"] for t in TERMS])
def test_term_heatbath_and_force(U0, term):
    ops = hmc.Ops(DIMS, U0, 1.0)
    eta = synth.gaussian_spinor(VH, 30)
    phi = hmc.heatbath(ops, term, eta)
    S = hmc.action(ops, term, phi, 1e-13)
    assert abs(S - np.vdot(eta, eta).real) < 1e-10 * S
    F = hmc.force(ops, term, phi, 1e-13)
    fun = lambda U: hmc.action(hmc.Ops(DIMS, U, 1.0), term, phi, 1e-13)
    for link, a in SAMPLES[:3]:
        ref = fd(fun, U0, link, a)
        assert abs(F[link // 4, link % 4, a] - ref) < 2e-6 * max(1, abs(ref))


HIGH_DEGREE = [dict(kind="polyq", kappa=0.120, n=62, n1=20, mu=1.2, nu=0.9),
               dict(kind="polycorr", kappa=0.120, n=20, mu=1.2, nu=0.9)]


@pytest.mark.parametrize("term", HIGH_DEGREE, ids=["polyq62_20", "polycorr20"])
def test_high_degree_filter_force(U0, term):
    """The filter nest's degrees (the quotient Q(62/20), a degree-20 correction): the forces
    still differentiate the actions.  The step of the differences is larger than above
    because a degree-62 product loses a few more digits of the action to rounding."""
    ops = hmc.Ops(DIMS, U0, 1.6)
    phi = hmc.heatbath(ops, term, synth.gaussian_spinor(VH, 30))
    F = hmc.force(ops, term, phi, 1e-13)
    fun = lambda U: hmc.action(hmc.Ops(DIMS, U, 1.6), term, phi, 1e-13)
    for link, a in SAMPLES[:3]:
        ref = fd(fun, U0, link, a, eps=3e-3)
        assert abs(F[link // 4, link % 4, a] - ref) < 1e-4 * abs(ref) + 1e-8


def test_polynomial_force_matrix_count(U0):
    """The incremental construction of eq. force_poly costs 2p - 2 K-mults (Table 3.2)."""
    g = json.load(open(os.path.join(GOLD, "poly_force_counts.json")))
    for p, want in zip(g["p"], g["mat_per_F1"]):
        calls = []

        class Counting:
            def K(self, v):
                calls.append(1)
                return v

        hmc._prod_vectors(Counting(), [0.5 + 0.1j] * p, 1.0, np.ones(3))
        assert len(calls) == want == 2 * p - 2


# ---------------------------------------------------------------- integrator

def test_link_update_exp(U0):
    P = synth.gaussian_momenta(V, 3)
    U = U0.copy()
    oracle.update_gauge(DIMS, 0.3, P, U)
    for l in (0, 77, 1023):
        x, mu = divmod(l, 4)
        Pm = sum(P[x, mu, a] * T[a] for a in range(8))
        want = sl.expm(0.3j * Pm) @ U0[x, mu]
        assert np.max(np.abs(U[x, mu] - want)) < 1e-14
    assert np.max(np.abs(np.einsum("xmab,xmcb->xmac", U, U.conj()) - np.eye(3))) < 1e-13
    assert np.max(np.abs(np.linalg.det(U) - 1)) < 1e-13
    oracle.update_gauge(DIMS, -0.3, P, U)
    assert np.max(np.abs(U - U0)) < 1e-14


def test_kinetic_term():
    P = synth.gaussian_momenta(V, 4)
    assert abs(oracle.kinetic(P) - 0.5 * np.sum(P * P)) < 1e-10


def _frac_or_lam(s, lam):
    s = s.replace("1-2lam", "X")
    if s == "lam":
        return lam
    if s == "X":
        return 1 - 2 * lam
    return Fraction(s)


def test_schedule_worked_example():
    g = json.load(open(os.path.join(GOLD, "schedule_demo.json")))
    lam = schedule.OMELYAN_LAMBDA
    inp = {k: [_frac_or_lam(s, lam) for s in v] for k, v in g["inputs"].items()}
    exp = {k: [_frac_or_lam(s, lam) for s in v] for k, v in g["expected"].items()}
    newT, newS = schedule.merge([inp["T1"], inp["T2"]], [inp["S1"], inp["S2"]])
    assert newT == exp["T"]
    assert newS[0] == exp["S1"]
    assert newS[1] == exp["S2"]
    assert schedule.is_symmetric(newT, newS)
    # the example's first scheme is the 3-step leapfrog and its second the 1-step 2MN
    T1, S1 = schedule.leapfrog(3)
    assert T1 == inp["T1"] and S1 == inp["S1"]
    T2, S2 = schedule.omelyan_2mn(1)
    assert T2 == inp["T2"] and S2 == [float(x) for x in inp["S2"]]


def _flow(newT, newS, sign, A, Bs):
    """The integrator's map for step sizes sign * (T', S'): T[t] = exp(t A), S_j[s] =
    exp(s B_j), applied in schedule order (each merged step: T then the S_j)."""
    M = np.eye(A.shape[0])
    for k, t in enumerate(newT):
        M = sl.expm(sign * float(t) * A) @ M
        for s, B in zip(newS, Bs):
            M = sl.expm(sign * s[k] * B) @ M
    return M


def _reversible(newT, newS):
    """Brute-force reversibility (App. B, time-step insertion theorem): running the
    schedule with negated steps undoes it, Phi(-h) Phi(h) = 1, for a time generator A that
    commutes with none of the space generators B_j, which commute among themselves (as
    the momentum updates S_j do) but are otherwise independent."""
    rng = np.random.default_rng(11)
    n = 5
    A = rng.standard_normal((n, n))
    A = A - A.T
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Bs = [Q @ np.diag(rng.standard_normal(n)) @ Q.T for _ in newS]
    M = _flow(newT, newS, -1.0, A, Bs) @ _flow(newT, newS, 1.0, A, Bs)
    return np.max(np.abs(M - np.eye(n))) < 1e-10


def test_is_symmetric_agrees_with_reversibility():
    """is_symmetric (the mirror condition) is True exactly for the schedules whose flow
    is undone by the negated flow: merged 2MN and leapfrog schemes, and False for each
    plausible defect (one term's space steps not mirrored, time steps not mirrored, a
    first-order scheme in the mix, a 1e-9 slip in one step)."""
    lam = schedule.OMELYAN_LAMBDA
    good = [schedule.merge(*zip(schedule.leapfrog(3), schedule.omelyan_2mn(1))),
            schedule.merge(*zip(*[schedule.omelyan_2mn(n) for n in (2, 3, 5)]))]
    bad = []
    T, S = good[0]
    bad.append((T, [S[0], [lam, 1 - 2 * lam, 0, 0, lam]]))                     # second row not mirrored
    bad.append(([Fraction(0), Fraction(1, 6), Fraction(1, 3), Fraction(1, 6), Fraction(1, 3)], S))  # times
    bad.append(schedule.merge([[0, Fraction(1)], schedule.omelyan_2mn(2)[0]],
                              [[1 / 3, 2 / 3], schedule.omelyan_2mn(2)[1]]))     # S[h/3] T[h] S[2h/3]
    T2, S2 = good[1]
    S2 = [list(r) for r in S2]
    k = next(i for i, v in enumerate(S2[1]) if v != 0)
    S2[1][k] += 1e-9
    bad.append((T2, S2))
    for T, S in good:
        assert _reversible(T, S) and schedule.is_symmetric(T, S)
    for T, S in bad:
        assert not _reversible(T, S)
        assert not schedule.is_symmetric(T, S)


@pytest.mark.parametrize("steps", [(10, 20, 40, 80), (10, 15, 40, 120), (3, 7, 11, 13)])
def test_schedule_sums_and_symmetry(steps):
    Ts, Ss = zip(*[schedule.omelyan_2mn(n) for n in steps])
    newT, newS = schedule.merge(Ts, Ss)
    assert sum(newT) == 1
    for s in newS:
        assert abs(sum(s) - 1.0) < 1e-13
    assert schedule.is_symmetric(newT, newS)
    # every step of every scheme appears, none twice
    for n, s in zip(steps, newS):
        assert sum(1 for v in s if v != 0) == 2 * n + 1


# ---------------------------------------------------------------- trajectories

def spec_cfg1(mult=1, terms=(0, 1, 2)):
    allt = [dict(kind="poly", kappa=0.110, n=4, mu=1.2, nu=0.9, steps=4),
            dict(kind="polycorr", kappa=0.110, n=4, mu=1.2, nu=0.9, steps=2),
            dict(kind="ratio", kappa_num=0.110, kappa_den=0.120, steps=1)]
    ts = [dict(allt[i]) for i in terms]
    for t in ts:
        t["steps"] *= mult
    return dict(dims=DIMS, beta=5.6, csw=1.0, kappa=0.120, gauge_steps=8 * mult, terms=ts)


def test_reversibility(U0):
    """Forward tau, negate P, forward tau again (the merged schedule is symmetric)
    returns to the start (App. B reversibility theorems)."""
    spec = spec_cfg1(1)
    P0 = synth.gaussian_momenta(V, 100)
    etas = [synth.gaussian_spinor(VH, 20 + i) for i in range(3)]
    ops = hmc.Ops(DIMS, U0, spec["csw"])
    phis = [hmc.heatbath(ops, t, e) for t, e in zip(spec["terms"], etas)]
    U, P = U0.copy(), P0.copy()
    hmc.md_evolve(spec, U, P, phis, 1e-13)
    assert np.max(np.abs(U - U0)) > 1e-2
    P = -P
    hmc.md_evolve(spec, U, P, phis, 1e-13)
    assert np.max(np.abs(U - U0)) < 1e-10
    assert np.max(np.abs(-P - P0)) < 1e-9


@pytest.mark.parametrize("terms", [(0,), (2,)], ids=["gauge+poly", "gauge+ratio"])
def test_dH_scales_as_h_squared(U0, terms):
    """Second-order integrator: scaling every step count by m gives dH ~ 1/m^2."""
    P = synth.gaussian_momenta(V, 100)
    etas = [synth.gaussian_spinor(VH, 20 + i) for i in range(3)]
    dH = []
    mults = [2, 4, 8]
    for m in mults:
        r = hmc.trajectory(spec_cfg1(m, terms=terms), U0, P, [etas[i] for i in terms], tol=1e-13)
        dH.append(abs(r["dH"]))
    slope = np.polyfit(np.log([1.0 / m for m in mults]), np.log(dH), 1)[0]
    assert abs(slope - 2) < 0.15, (dH, slope)


@pytest.mark.slow
def test_exp_minus_dH_average_quenched():
    """<exp(-dH)> = 1 (within 3 sigma) over 200 quenched trajectories on 4^4."""
    U = synth.random_gauge(DIMS, seed=1, spread=0.5)
    vals = []
    for traj in range(200):
        spec = dict(dims=DIMS, beta=5.6, csw=0.0, kappa=0.12, gauge_steps=6, terms=[])
        P = synth.gaussian_momenta(V, 1000 + traj)
        r = hmc.trajectory(spec, U, P, [], u=synth.uniform(5000 + traj)[0])
        vals.append(math.exp(-r["dH"]))
        if r["accept"]:
            U = r["U"]
    m = np.mean(vals)
    err = np.std(vals) / math.sqrt(len(vals))
    assert abs(m - 1) < 3 * err + 1e-3, (m, err)


def test_schedule_with_det_row_sums_to_tau():
    """With S_det on its own scale the merged schedule has one more row; every
    row's space steps and the time steps each add up to tau (App. B)."""
    spec = dict(dims=(4, 4, 4, 4), gauge_steps=8, terms=[dict(steps=2), dict(steps=4)], det_steps=3, tau=1.0)
    T, S = hmc.build_schedule(spec)
    assert len(S) == 4
    assert abs(sum(float(t) for t in T) - 1.0) < 1e-12
    for row in S:
        assert abs(sum(float(s) for s in row) - 1.0) < 1e-12
    assert sum(1 for s in S[3] if s != 0) == 2 * 3 + 1  # 2MN, 3 steps: 2n + 1 space steps after merging
