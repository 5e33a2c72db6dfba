"""Generalized multi-scale integrator schedule (paper App. B).

TEST INFRASTRUCTURE ONLY (part of the oracle).

Each action term j has its own symplectic scheme written as two equal-length lists:
T_j (time steps, the first one 0) and S_j (space steps), enacted as
T[0] S[0] T[1] S[1] ...  The generalized integrator superimposes the schemes on
the common time axis (the time-step insertion operator, eq. uber_gen) and the
merge follows the example algorithm of App. B "Implementation": advance by the
smallest pending time step; a scheme whose pending step ends there contributes its
next space step, every other scheme contributes a zero space step and has its
pending time step shortened.

Time steps are exact rationals (fractions.Fraction) so that coincident insertion
times compare equal; space steps are carried through unchanged.
"""
from fractions import Fraction

# Minimum-norm parameter of the second-order Omelyan integrator (Omelyan, Mryglod,
# Folk 2003), the paper's 2MN scheme (eq. 2MNSTS).
OMELYAN_LAMBDA = 0.1931833275037836


def omelyan_2mn(nsteps, tau=Fraction(1), lam=OMELYAN_LAMBDA):
    """n-step 2MN space-time-space scheme S[lh] T[h/2] S[(1-2l)h] T[h/2] S[lh], h = tau/n,
    with the adjacent space steps of consecutive steps merged (S[a]S[b] = S[a+b])."""
    h = Fraction(tau) / nsteps
    T = [Fraction(0)]
    S = [lam * float(h)]
    for k in range(nsteps):
        T.append(h / 2)
        S.append((1 - 2 * lam) * float(h))
        T.append(h / 2)
        S.append((2 * lam if k < nsteps - 1 else lam) * float(h))
    return T, S


def leapfrog(nsteps, tau=Fraction(1)):
    """n-step leapfrog S[h/2] T[h] S[h/2] ... with merged adjacent space steps."""
    h = Fraction(tau) / nsteps
    T = [Fraction(0)] + [h] * nsteps
    S = [h / 2] + [h] * (nsteps - 1) + [h / 2]
    return T, S


def merge(T_lists, S_lists):
    """Merge per-term (T_j, S_j) lists into (T', [S'_j]) per App. B.

    Returns the merged time steps and, per term, the space step at each merged
    position (0 where the term does nothing)."""
    T_lists = [list(map(Fraction, t)) for t in T_lists]
    S_lists = [list(s) for s in S_lists]
    total = sum(T_lists[0])
    for t in T_lists:
        if sum(t) != total:
            raise ValueError("all schemes must span the same trajectory length")
        if len(t) == 0:
            raise ValueError("empty scheme")
    for t, s in zip(T_lists, S_lists):
        if len(t) != len(s):
            raise ValueError("T and S lists of a scheme must have equal length")
    n = len(T_lists)
    new_T = []
    new_S = [[] for _ in range(n)]
    tau = Fraction(0)
    first = True
    while first or tau < total:
        first = False
        d_tau = min(t[0] for t in T_lists)
        new_T.append(d_tau)
        for i in range(n):
            if T_lists[i][0] == d_tau:
                new_S[i].append(S_lists[i].pop(0))
                T_lists[i].pop(0)
            else:
                new_S[i].append(0)
                T_lists[i][0] -= d_tau
        tau += d_tau
    for t in T_lists:
        if t:
            raise ValueError("schemes did not end together")
    return new_T, new_S


def is_symmetric(new_T, new_S):
    """Mirror condition of the App. B reversibility theorem: the schedule read
    backwards gives the same space steps (term by term) at mirrored times."""
    n = len(new_T)
    times = []
    t = Fraction(0)
    for d in new_T:
        t += d
        times.append(t)
    total = times[-1]
    for k in range(n):
        if times[k] + times[n - 1 - k] != total:
            return False
        for s in new_S:
            if abs(s[k] - s[n - 1 - k]) > 1e-15 * max(1.0, abs(s[k])):
                return False
    return True
