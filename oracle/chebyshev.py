"""Chebyshev polynomial filter scalars (paper App. A; pole residues from App. C).

TEST INFRASTRUCTURE ONLY (part of the oracle).

P_n(z) = a_n prod_{k=1..n} (z - z_k) approximates 1/z, with
  z_k = mu (1 - cos th_k) - i sqrt(mu^2 - nu^2) sin th_k,  th_k = 2 pi k / (n + 1),
  a_n = 1 / (mu prod_k (mu - z_k)).
Partial fractions of prod 1/(z - z_i) over the n roots plus z_{n+1} = 0 give the
residues r_i = prod_{j != i} 1/(z_j - z_i) (App. C, polynomial correction force).
"""
import math


def roots(n, mu, nu):
    """The n roots z_1..z_n in the paper's order k = 1..n."""
    b = math.sqrt(mu * mu - nu * nu)
    out = []
    for k in range(1, n + 1):
        th = 2.0 * math.pi * k / (n + 1)
        out.append(complex(mu * (1.0 - math.cos(th)), -b * math.sin(th)))
    return out


def norm(n, mu, nu):
    """a_n = 1 / (mu * prod_k (mu - z_k))."""
    p = complex(mu)
    for z in roots(n, mu, nu):
        p *= (mu - z)
    return 1.0 / p


def quotient(n, n1, mu, nu):
    """Q = P_n / P_n1 for two filters on the same ellipse with (n1 + 1) dividing (n + 1)
    (App. A): the roots of P_n that are not roots of P_n1, found by comparing values,
    in the paper's order, and the norm a_n / a_n1.  Q has degree n - n1 (eq. 2poly)."""
    if n1 <= 0 or n1 >= n or (n + 1) % (n1 + 1):
        raise ValueError("P_n1 divides P_n only when (n1 + 1) divides (n + 1)")
    inner = roots(n1, mu, nu)
    scale = max(mu, 1.0)
    keep = [z for z in roots(n, mu, nu) if min(abs(z - w) for w in inner) > 1e-9 * scale]
    if len(keep) != n - n1:
        raise ValueError("root sets do not nest")
    return keep, norm(n, mu, nu) / norm(n1, mu, nu)


def evaluate(z, n, mu, nu):
    """P_n(z) by its product form."""
    v = norm(n, mu, nu)
    for r in roots(n, mu, nu):
        v *= (z - r)
    return v


def residues(zs):
    """r_i = prod_{j != i} 1 / (z_j - z_i) for the given list of distinct poles."""
    out = []
    for i, zi in enumerate(zs):
        p = complex(1.0)
        for j, zj in enumerate(zs):
            if j != i:
                p *= 1.0 / (zj - zi)
        out.append(p)
    return out


def conjugate_partner(zs, tol=1e-12):
    """For each pole, the index of its complex conjugate in the list (App. C)."""
    out = []
    for zi in zs:
        best = min(range(len(zs)), key=lambda j: abs(zs[j] - zi.conjugate()))
        if abs(zs[best] - zi.conjugate()) > tol * max(1.0, abs(zi)):
            raise ValueError("pole set is not closed under conjugation")
        out.append(best)
    return out


def divides(p1, p2, mu, nu, tol=1e-12):
    """True when every root of P_{p1} is a root of P_{p2} (same mu, nu)."""
    r2 = roots(p2, mu, nu)
    return all(min(abs(z - w) for w in r2) < tol for z in roots(p1, mu, nu))
