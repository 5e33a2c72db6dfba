"""Seeded synthetic inputs shared by the library's callers and the oracle.

This module holds none of the method's arithmetic: it only draws random numbers
and shapes them into fields in the canonical layouts.  Random numbers that the
method itself draws (momenta, pseudofermion noise, the Metropolis uniform) are
drawn here and passed in as inputs.

Canonical layouts (numpy):
  gauge    U[V, 4, 3, 3] complex128, lexicographic sites (x fastest), mu = x,y,z,t
  spinor   psi[Vh, 4, 3] complex128 on one parity (even-odd index = lex // 2)
  momenta  P[V, 4, 8] float64, coefficients of T_a = lambda_a / 2
Each purpose has its own numpy PCG64 stream with a fixed draw order.
"""
import numpy as np


def volume(dims):
    return int(np.prod(dims))


def _reunitarise(U):
    """Gram-Schmidt on rows 1-2 and row 3 = conj(row1 x row2): an SU(3) matrix."""
    r0 = U[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def random_gauge(dims, seed=0, spread=0.2):
    """U = exp(i * spread * H) per link, H traceless Hermitian with N(0,1) entries
    (per site in lexicographic order and mu = 0..3: 3 diagonal entries, then Re and
    Im of the 3 upper off-diagonal entries), reunitarised to SU(3)."""
    V = volume(dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((V, 4, 9))
    H = np.zeros((V, 4, 3, 3), np.complex128)
    for i in range(3):
        H[..., i, i] = g[..., i]
    off = [(0, 1), (0, 2), (1, 2)]
    for k, (i, j) in enumerate(off):
        H[..., i, j] = g[..., 3 + 2 * k] + 1j * g[..., 4 + 2 * k]
        H[..., j, i] = np.conj(H[..., i, j])
    tr = np.trace(H, axis1=-2, axis2=-1) / 3.0
    for i in range(3):
        H[..., i, i] -= tr
    w, v = np.linalg.eigh(H)
    U = np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * spread * w), np.conj(v))
    return np.ascontiguousarray(_reunitarise(U))


def unit_gauge(dims):
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), np.complex128)
    for i in range(3):
        U[..., i, i] = 1.0
    return U


def random_su3(n, seed):
    """n Haar-distributed SU(3) matrices (QR of complex Gaussian matrices)."""
    rng = np.random.default_rng(seed)
    Z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2)
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    Q[:, :, 2] /= det[:, None]
    return np.ascontiguousarray(Q)


def gaussian_spinor(Vh, seed, nfield=None):
    """Complex Gaussian spinor field(s) with density exp(-eta^dag eta):
    Re and Im ~ N(0, 1/2)."""
    rng = np.random.default_rng(seed)
    shape = (Vh, 4, 3) if nfield is None else (nfield, Vh, 4, 3)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return np.ascontiguousarray((re + 1j * im) / np.sqrt(2.0))


def gaussian_momenta(V, seed):
    """Momentum coefficients p_a ~ N(0, 1) per link (density exp(-sum tr P^2))."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((V, 4, 8)))


def uniform(seed, n=1):
    rng = np.random.default_rng(seed)
    return rng.random(n)


def network_weights(seed, scale=0.1, nin=4, nhid=12):
    """Initial weights of the parallel-transport convolution network: complex
    N(0, 2 scale^2) entries for the two transport layers [8][nhid][nin] and
    [8][nin][nhid], and the identity for the site-local skip term [nin][nin] (so
    the network starts close to the identity preconditioner)."""
    rng = np.random.default_rng(seed)
    c = lambda *s: (rng.standard_normal(s) + 1j * rng.standard_normal(s)) * scale
    return c(8, nhid, nin), c(8, nin, nhid), np.eye(nin, dtype=np.complex128)
