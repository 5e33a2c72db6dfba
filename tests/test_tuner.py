"""Step-size tuning helpers (paper Sec. 2.4 eq. force_tune, Sec. 3 eqs. cost_func and
error_corrected): the host arithmetic, pinned against direct numerical integration
and the defining relations."""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_1609_02652_amd import tuner


@pytest.mark.parametrize("m", [0.05, 0.3, 1.0, 3.0])
def test_acceptance_from_dH_is_gaussian_average(m):
    """For dH ~ N(m, 2m) (the Gaussian with <exp(-dH)> = 1), <min(1, exp(-dH))> by quadrature."""
    s = math.sqrt(2 * m)
    pdf = lambda x: math.exp(-(x - m) ** 2 / (2 * s * s)) / (s * math.sqrt(2 * math.pi))
    lo, hi = m - 30 * s, m + 30 * s
    mean_exp = integrate.quad(lambda x: math.exp(-x) * pdf(x), lo, hi, limit=200)[0]
    assert abs(mean_exp - 1) < 1e-9
    acc = integrate.quad(lambda x: min(1.0, math.exp(-x)) * pdf(x), lo, hi, points=[0.0], limit=200)[0]
    assert abs(tuner.acceptance_from_dH(m) - acc) < 1e-7


def test_dH_for_acceptance_inverts():
    for p in (0.5, 0.65, 0.7, 0.75, 0.9):
        assert abs(tuner.acceptance_from_dH(tuner.dH_for_acceptance(p)) - p) < 1e-10


def test_balanced_steps_keep_force_times_step_constant():
    f = [40.0, 3.1, 0.9, 0.2]
    for c in (0.05, 0.13, 1.0):
        n = tuner.balanced_steps(f, c, tau=1.0)
        for fi, ni in zip(f, n):
            h = 1.0 / ni
            assert fi * h <= c + 1e-15                        # never coarser than c
            assert ni == 1 or fi / (ni - 1) > c               # the coarsest step with fi h <= c
    assert tuner.balanced_steps([1e-9], 1.0) == [1]


def test_corrected_error_and_cost():
    v = np.array([3.0, 5.0, 4.0, 6.0, 2.0])
    want = math.sqrt(2 * 12.5) * np.std(v, ddof=1) / math.sqrt(5)
    assert abs(tuner.corrected_error(v) - want) < 1e-14
    nmat, acc = [100.0, 110.0, 90.0, 100.0], [1, 0, 1, 1]
    c, dc = tuner.cost(nmat, acc)
    assert abs(c - 100.0 / 0.75) < 1e-12
    rel = math.hypot(tuner.corrected_error(nmat) / 100.0, tuner.corrected_error(acc) / 0.75)
    assert abs(dc - c * rel) < 1e-12
    assert tuner.cost([1.0, 1.0], [0, 0])[0] == float("inf")


def test_mean_dH_estimate_matches_gaussian_model():
    """For dH ~ N(m, 2m), <dH^2> / 2 = m + m^2 / 2 -> m for small m; on a large sample the
    estimate is within a few per cent of m + m^2 / 2 and always positive."""
    rng = np.random.default_rng(3)
    for m in (0.1, 0.3):
        x = rng.normal(m, math.sqrt(2 * m), size=200000)
        assert abs(tuner.mean_dH_estimate(x) - (m + m * m / 2)) < 0.03 * m
    assert tuner.mean_dH_estimate([-0.5, 0.2]) > 0


class _ModelTuner(tuner.StepTuner):
    """The search of StepTuner.tune against a model chain: <dH> = m*(c) exactly, with the h^4
    law below 1.4 c* and a steep rise above it (the coarse steps leaving the stable range)."""

    def __init__(self, c_star):
        self.c_star, self.tau, self.calls = c_star, 1.0, []

    def run(self, steps, ntraj):
        c = self.c_cur
        x = c / self.c_star
        m = tuner.dH_for_acceptance(0.70) * (x ** 4 if x < 1.4 else 1.4 ** 4 * math.exp(20 * (x - 1.4)))
        self.calls.append(c)
        return [(math.sqrt(2 * m), 1, 100)] * ntraj


def test_tune_search_reaches_the_acceptance_window(monkeypatch):
    real = tuner.balanced_steps
    for c_star, c0 in ((0.15, 0.30), (0.15, 0.02), (1.0, 0.9)):
        T = _ModelTuner(c_star)

        def fake_balanced(fmax, c, tau=1.0, T=T):
            T.c_cur = c
            return real(fmax, c, tau)
        monkeypatch.setattr(tuner, "balanced_steps", fake_balanced)
        hist, best = T.tune([1.0, 2.0], c0, ntraj=2, rounds=8)
        m = tuner.mean_dH_estimate([t[0] for t in hist[best][2]])
        assert tuner.ACC_RANGE[0] <= tuner.acceptance_from_dH(m) <= tuner.ACC_RANGE[1], (c_star, c0, T.calls)


def test_tau_int_of_an_ar1_chain():
    """tau_int of an AR(1) chain x_t = phi x_{t-1} + e_t is (1 + phi) / (2 (1 - phi)) in the
    convention sigma = sqrt(2 tau_int) sigma_p / sqrt(N); uncorrelated noise gives 1/2."""
    rng = np.random.default_rng(3)
    for phi in (0.0, 0.5, 0.8):
        n = 200000
        e = rng.standard_normal(n)
        x = np.empty(n)
        x[0] = e[0]
        for t in range(1, n):
            x[t] = phi * x[t - 1] + e[t]
        want = (1 + phi) / (2 * (1 - phi))
        got = tuner.tau_int(x)
        assert abs(got - want) < 0.06 * want + 0.02, (phi, got, want)
