"""Degenerate and boundary cases of the C-ABI on the GPU: a zero right-hand side in
every solver (the answer is x = 0 with no division by |b| = 0), kappa = 0 (Mhat = A_ee),
the degree-0 filter (norm * in), a single real shift, and argument errors reported as
error codes before any launch."""
import numpy as np
import pytest

import oracle
from paper_1609_02652_amd import synth

pytestmark = pytest.mark.gpu

DIMS = (6, 4, 4, 8)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.fixture(scope="module")
def setup():
    from paper_1609_02652_amd.pfmp import Lattice
    print("case", DIMS, flush=True)
    U = synth.random_gauge(DIMS, seed=8)
    lat = Lattice(DIMS)
    lat.set_gauge(U)
    lat.set_operator(0, 0.125, 1.3)
    lat.set_operator(1, 0.0, 1.3)
    yield U, lat
    lat.close()


def test_zero_source_every_solver(setup):
    from paper_1609_02652_amd.pfmp import F32, F16
    U, lat = setup
    zero = lat.field()
    for prec in (None, F32, F16):
        x, st = lat.cg_solve(0, zero, maxiter=50) if prec is None else lat.cg_solve(0, zero, prec=prec, maxiter=50)
        xs = lat.spinor_numpy(x)
        assert np.all(np.isfinite(xs)) and np.max(np.abs(xs)) == 0.0 and st["true_res"] == 0.0, prec
    xs, st = lat.cg_multishift(0, [0.5 + 0.2j, 0.0], zero, maxiter=50)
    for x in xs:
        assert np.max(np.abs(lat.spinor_numpy(x))) == 0.0
    b = lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 3))
    sols, sts = lat.cg_solve_batch([0, 0], [zero, b], maxiter=500)
    assert np.max(np.abs(lat.spinor_numpy(sols[0]))) == 0.0 and sts[0]["iters"] == 0
    assert sts[1]["true_res"] <= 1e-10
    for W in (None, synth.network_weights(1, scale=0.1)):
        x, st = lat.fcg_solve(0, W, zero, maxiter=50)
        assert np.max(np.abs(lat.spinor_numpy(x))) == 0.0 and st["true_res"] == 0.0


def test_kappa_zero_is_the_even_clover_term(setup):
    U, lat = setup
    psi = synth.gaussian_spinor(lat.Vh, 4)
    x = lat.pack_spinor(psi)
    got = lat.spinor_numpy(lat.apply_M(1, x))
    assert rel(got, lat.spinor_numpy(lat.apply_clover(1, 0, False, x))) < 1e-15
    assert rel(got, oracle.Operator(DIMS, U, 0.0, 1.3).M(psi)) < 1e-12


def test_degree_zero_filter_and_single_shift(setup):
    U, lat = setup
    psi = synth.gaussian_spinor(lat.Vh, 5)
    x = lat.pack_spinor(psi)
    out = lat.apply_poly(0, [], 0.5 - 2j, x)
    assert rel(lat.spinor_numpy(out), (0.5 - 2j) * psi) < 1e-15
    # one real shift: (Khat + 0.3) x = b, residual checked with the oracle's operator
    xs, st = lat.cg_multishift(0, [-0.3], x, tol=1e-11)
    xg = lat.spinor_numpy(xs[0])
    op = oracle.Operator(DIMS, U, 0.125, 1.3)
    assert rel(op.K(xg) + 0.3 * xg, psi) < 1e-10


def test_argument_errors(setup):
    from paper_1609_02652_amd.pfmp import PfmpError
    U, lat = setup
    x = lat.field()
    with pytest.raises(PfmpError) as e:
        lat.apply_M(7, x)                       # slot never configured
    assert e.value.code in (-1, -5)
    with pytest.raises(PfmpError) as e:
        lat.apply_M(99, x)                      # slot out of range
    assert e.value.code == -1
    with pytest.raises(PfmpError) as e:
        lat.cg_multishift(0, [0.1] * 200, x)    # more shifts than supported
    assert e.value.code == -1
    with pytest.raises(PfmpError) as e:
        lat.cg_solve_batch([0] * 9, [x] * 9)    # more than 8 right-hand sides
    assert e.value.code == -1


def test_spec_errors_and_force_norms_without_det(setup):
    """An intermediate filter whose inner degree does not divide the outer one ((4 + 1) does
    not divide (8 + 1)), an inner degree equal to the outer one and an odd degree are rejected
    before any work;
    with det_op < 0 the S_det row of the force sizes is zero and the gauge row is positive."""
    from paper_1609_02652_amd.pfmp import PfmpError
    U, lat = setup
    bad = [[dict(kind="polyq", op=0, n=8, n1=4, mu=1.2, nu=0.9, steps=2)],
           [dict(kind="polyq", op=0, n=8, n1=8, mu=1.2, nu=0.9, steps=2)],
           [dict(kind="poly", op=0, n=5, mu=1.2, nu=0.9, steps=2)]]
    phi = [lat.field()]
    for terms in bad:
        with pytest.raises(PfmpError) as e:
            lat.force_norms(lat.spec(5.6, terms, 4), phi)
        assert e.value.code == -1
    sp = lat.spec(5.6, [dict(kind="polyq", op=0, n=8, n1=2, mu=1.2, nu=0.9, steps=2)], 4, det_op=-1)
    phi = [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 5))]
    F = lat.force_norms(sp, phi)
    assert F.shape == (3, 2)
    assert np.all(F[:2] > 0) and np.all(F[2] == 0)
