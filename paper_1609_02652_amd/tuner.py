"""Step-size tuning and cost of an action (paper Sec. 2.4 and 3).

Host-side control only: every force, heatbath and trajectory runs in the library
(``Lattice.force_norms``, ``Lattice.trajectory``); random inputs come from the seeded
generators of ``synth``.

* Forces: each row of the schedule (gauge action, every term, S_det on its own scale)
  is sized by its maximal force over links, averaged over the start fields of a few
  trajectories; the maximal rather than the mean force is the paper's choice, as it
  captures part of the force variance (Sec. 2.4).
* Balance: step sizes with F_i h_i = const (eq. force_tune), i.e. n_i = ceil(tau F_i / c)
  2MN steps, with one free scale c.
* Acceptance: c is tuned so that P_acc lies in [0.65, 0.75] (Sec. 3, cost-effective for a
  second-order integrator).  For Gaussian dH with <exp(-dH)> = 1, <dH> = <dH^2> / 2 and
  P_acc = erfc(sqrt(<dH>) / 2); the mean is estimated as <dH^2> / 2, which a few
  trajectories give far more stably than the mean of dH itself (that can come out
  negative).  <dH> scales as h^4 for a second-order integrator, so a round rescales c by
  (dH_target / <dH>)^(1/4), limited to a factor 1.6 either way, until one c too fine and
  one too coarse are known; then c is bisected geometrically between them (near the
  stability limit of the coarse steps dH grows much faster than h^4).
* Cost: C = N_mat / P_acc (eq. cost_func) with N_mat the K-multiplications per
  trajectory; errors sqrt(2 tau_int) sigma_p / sqrt(N) (eq. error_corrected) with the
  paper's tau_int = 12.5 by default, or tau_int measured on the chain itself (tau_int(),
  self-consistent window), propagated to C.
"""
import math

import numpy as np

from . import synth

TAU_INT = 12.5
ACC_RANGE = (0.65, 0.75)


def acceptance_from_dH(mean_dH):
    """P_acc = erfc(sqrt(<dH>) / 2) for Gaussian dH with <exp(-dH)> = 1."""
    return math.erfc(math.sqrt(max(mean_dH, 0.0)) / 2.0)


def dH_for_acceptance(p):
    """The <dH> at which acceptance_from_dH gives p (bisection)."""
    lo, hi = 0.0, 50.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if acceptance_from_dH(mid) > p:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def mean_dH_estimate(dH):
    """<dH> estimated as <dH^2> / 2 (Gaussian dH with <exp(-dH)> = 1)."""
    return 0.5 * float(np.mean(np.square(dH)))


def balanced_steps(fmax, c, tau=1.0):
    """2MN step counts with F_i h_i = c (h_i = tau / n_i), at least one step each."""
    return [max(1, int(math.ceil(tau * f / c))) for f in fmax]


def corrected_error(values, tau_int=TAU_INT):
    """sigma = sqrt(2 tau_int) sigma_p / sqrt(N) (eq. error_corrected)."""
    v = np.asarray(values, dtype=float)
    if len(v) < 2:
        return float("nan")
    return math.sqrt(2.0 * tau_int) * float(np.std(v, ddof=1)) / math.sqrt(len(v))


def tau_int(series, c=5.0):
    """Integrated autocorrelation time tau_int = 1/2 + sum_{t>=1} rho(t) of a Markov-chain
    series (the convention of eq. error_corrected: sigma = sqrt(2 tau_int) sigma_p / sqrt(N)),
    summed up to the first window W >= c tau_int(W) (self-consistent window)."""
    v = np.asarray(series, dtype=float)
    n = len(v)
    if n < 4:
        return float("nan")
    d = v - v.mean()
    var = float(np.dot(d, d)) / n
    if var == 0:
        return 0.5
    tau = 0.5
    for w in range(1, n // 2):
        tau += float(np.dot(d[:-w], d[w:])) / (n * var)
        if w >= c * tau:
            return tau
    return tau


def cost(nmat, accepts, tau_int=TAU_INT):
    """C = <N_mat> / P_acc with its corrected error (relative errors added in quadrature)."""
    n, a = float(np.mean(nmat)), float(np.mean(accepts))
    if a == 0:
        return float("inf"), float("nan")
    c = n / a
    rel = math.hypot(corrected_error(nmat, tau_int) / n, corrected_error(accepts, tau_int) / a)
    return c, c * rel


class StepTuner:
    """Tune the 2MN step counts of one action on a lattice.

    build(steps) must return an HMC spec for the row step counts ``steps`` = [gauge,
    term 1 .. term n, S_det] (S_det ignored when the action has no det row)."""

    def __init__(self, lat, build, nterms, tau=1.0, seed=5000):
        self.lat, self.build, self.nterms, self.tau, self.seed = lat, build, nterms, tau, seed
        self.k = 0

    def _inputs(self):
        lat, k = self.lat, self.k
        self.k += 1
        P = lat.pack_momenta(synth.gaussian_momenta(lat.V, self.seed + k))
        etas = [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, self.seed + 100000 + 8 * k + j))
                for j in range(self.nterms)]
        return P, etas, synth.uniform(self.seed + 200000 + k)[0]

    def measure_forces(self, steps, ntraj):
        """Mean over the start fields of ntraj trajectories (run with ``steps``, accepted
        or rejected as drawn) of each row's (max, mean) force."""
        rows = []
        sp = self.build(steps)
        for _ in range(ntraj):
            P, etas, u = self._inputs()
            phis = self.lat.heatbath(sp, etas)
            rows.append(self.lat.force_norms(sp, phis))
            self.lat.trajectory(sp, P, etas, u)
        return np.mean(rows, axis=0)

    def run(self, steps, ntraj):
        """ntraj trajectories of the Markov chain with ``steps``: dH, accepts, K-mults."""
        sp = self.build(steps)
        out = []
        for _ in range(ntraj):
            P, etas, u = self._inputs()
            st = self.lat.trajectory(sp, P, etas, u)
            out.append((st["dH"], int(st["accept"]), st["kmults"]))
        return out

    def tune(self, fmax, c0, ntraj=8, rounds=5, target=0.70):
        """Search c until the P_acc estimate lies in ACC_RANGE.  Returns the rounds as
        (c, steps, trajectories) and the index of the round whose estimate is closest to
        the target (the tuned choice)."""
        dH_t = dH_for_acceptance(target)
        c, hist = c0, []
        fine, coarse = None, None     # largest c found too accurate, smallest found too coarse
        for _ in range(rounds):
            steps = balanced_steps(fmax, c, self.tau)
            traj = self.run(steps, ntraj)
            hist.append((c, steps, traj))
            m = mean_dH_estimate([t[0] for t in traj])
            p = acceptance_from_dH(m)
            if ACC_RANGE[0] <= p <= ACC_RANGE[1]:
                break
            if p > ACC_RANGE[1]:
                fine = c if fine is None else max(fine, c)
            else:
                coarse = c if coarse is None else min(coarse, c)
            if fine is not None and coarse is not None:
                c = math.sqrt(fine * coarse)
            else:
                c *= min(1.6, max(1 / 1.6, (dH_t / max(m, 1e-12)) ** 0.25))
        best = min(range(len(hist)),
                   key=lambda k: abs(math.log(max(mean_dH_estimate([t[0] for t in hist[k][2]]), 1e-12) / dH_t)))
        return hist, best
