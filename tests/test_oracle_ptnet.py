"""Pins for the oracle's learned-preconditioner network and flexible CG (CPU).

The analytic gradients are checked by central finite differences of the loss;
the network by gauge covariance N(U^W, W r) = W N(U, r); flexible CG with the
identity by plain CG's iteration count and solution."""
import numpy as np
import pytest

import oracle
from oracle import ptnet
from paper_1609_02652_amd import synth

DIMS = (4, 4, 4, 4)


def coords(dims, lex):
    c = []
    for L in dims:
        c.append(lex % L)
        lex //= L
    return c


@pytest.fixture(scope="module")
def setup():
    U = synth.random_gauge(DIMS, seed=2)
    net = ptnet.PTNet(DIMS, U)
    op = oracle.Operator(DIMS, U, 0.12, 1.0)
    W = ptnet.init_weights(3, scale=0.3)
    rs = [synth.gaussian_spinor(128, 40 + k) for k in range(2)]
    pairs = [(op.K(e), e) for e in [synth.gaussian_spinor(128, 50 + k) for k in range(2)]]
    return U, net, op, W, rs, pairs


def test_gradients_match_finite_differences(setup):
    U, net, op, W, rs, pairs = setup
    loss, A1, A2, A0 = net.grads(pairs, *W)
    assert abs(loss - net.loss(pairs, *W)) < 1e-12 * loss
    rng = np.random.default_rng(0)
    for which, A in ((0, A1), (1, A2), (2, A0)):
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in W[which].shape)
            for part, dirv in (("re", 1.0), ("im", 1j)):
                eps = 1e-6
                Wp = [w.copy() for w in W]
                Wm = [w.copy() for w in W]
                Wp[which][idx] += eps * dirv
                Wm[which][idx] -= eps * dirv
                fd = (net.loss(pairs, *Wp) - net.loss(pairs, *Wm)) / (2 * eps)
                # dL = 2 Re(A dW): dW = eps -> 2 Re A, dW = i eps -> -2 Im A
                an = 2 * A[idx].real if part == "re" else -2 * A[idx].imag
                assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (which, idx, part, fd, an)


def test_residual_objective_gradients_match_finite_differences(setup):
    """The preconditioned-residual objective sum |K z(rhat) - rhat|^2 (K = Khat of
    the oracle operator): analytic gradient against central differences."""
    U, net, op, W, rs, pairs = setup
    K = lambda v: op.K(v)
    loss, A1, A2, A0 = net.grads(rs, *W, K=K)
    # the loss written out independently: |K N(r)/|r| - r/|r||^2
    direct = sum(np.linalg.norm(K(net.apply(r, *W)) - r) ** 2 / np.linalg.norm(r) ** 2 for r in rs)
    assert abs(loss - direct) < 1e-10 * direct
    rng = np.random.default_rng(1)
    for which, A in ((0, A1), (1, A2), (2, A0)):
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in W[which].shape)
            for part, dirv in (("re", 1.0), ("im", 1j)):
                eps = 1e-6
                Wp = [w.copy() for w in W]
                Wm = [w.copy() for w in W]
                Wp[which][idx] += eps * dirv
                Wm[which][idx] -= eps * dirv
                fd = (net.loss(rs, *Wp, K=K) - net.loss(rs, *Wm, K=K)) / (2 * eps)
                an = 2 * A[idx].real if part == "re" else -2 * A[idx].imag
                assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (which, idx, part, fd, an)


def test_network_is_gauge_covariant(setup):
    U, net, op, W, rs, pairs = setup
    V = 256
    Om = synth.random_su3(V, seed=9)
    lexeo, _, _ = oracle.index_maps(DIMS)
    Ug = np.empty_like(U)
    for x in range(V):
        c = coords(DIMS, x)
        for mu in range(4):
            d = list(c)
            d[mu] = (d[mu] + 1) % DIMS[mu]
            y = d[0] + DIMS[0] * (d[1] + DIMS[1] * (d[2] + DIMS[2] * d[3]))
            Ug[x, mu] = Om[x] @ U[x, mu] @ Om[y].conj().T
    netg = ptnet.PTNet(DIMS, Ug)
    r = rs[0]
    Oe = Om[lexeo[0]]
    rot = lambda f: np.einsum("iab,isb->isa", Oe, f)
    assert np.max(np.abs(netg.apply(rot(r), *W) - rot(net.apply(r, *W)))) < 1e-12


def test_network_is_homogeneous(setup):
    U, net, op, W, rs, pairs = setup
    r = rs[1]
    assert np.max(np.abs(net.apply(3.7 * r, *W) - 3.7 * net.apply(r, *W))) < 1e-12


def test_flexible_cg_identity_is_cg(setup):
    U, net, op, W, rs, pairs = setup
    b = rs[0]
    x, k = ptnet.flexible_cg(op.K, lambda v: v.copy(), b, 1e-11)
    xo, st = op.cg(b, tol=1e-11)
    assert abs(k - st["iters"]) <= 1
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-9


def test_flexible_cg_with_network_converges(setup):
    U, net, op, W, rs, pairs = setup
    b = rs[1]
    x, k = ptnet.flexible_cg(op.K, lambda v: net.apply(v, *W), b, 1e-10, maxiter=2000)
    assert np.linalg.norm(op.K(x) - b) / np.linalg.norm(b) < 1e-10
