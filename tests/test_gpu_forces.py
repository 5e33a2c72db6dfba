"""GPU parity of the polynomial filter, forces and integrator steps against the
FP64 oracle (through the C-ABI).  The oracle differentiates the definitions by
the product rule; the library uses spin-projected outer products and clover-leaf
insertions, so agreement checks one against the other."""
import numpy as np
import pytest

import oracle
from oracle import chebyshev
from paper_1609_02652_amd import synth

pytestmark = pytest.mark.gpu

DIMS = [(6, 4, 4, 8), (6, 6, 4, 6)]


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.fixture(scope="module", params=DIMS, ids=lambda d: "x".join(map(str, d)))
def setup(request):
    from paper_1609_02652_amd.pfmp import Lattice
    dims = request.param
    print("case", dims, flush=True)
    U = synth.random_gauge(dims, seed=4)
    lat = Lattice(dims)
    lat.set_gauge(U)
    ops = {0: (0.1240, 1.25), 1: (0.1300, 0.0)}
    for k, (kap, csw) in ops.items():
        lat.set_operator(k, kap, csw)
    oops = {k: oracle.Operator(dims, U, kap, csw) for k, (kap, csw) in ops.items()}
    yield dims, U, lat, oops
    lat.close()


def test_apply_poly_and_chain(setup):
    from paper_1609_02652_amd import pfmp
    dims, U, lat, ops = setup
    z, a = pfmp.chebyshev(6, 1.2, 0.9)
    psi = synth.gaussian_spinor(lat.Vh, 20)
    f = lat.pack_spinor(psi)
    chain = [lat.field() for _ in range(6)]
    out = lat.apply_poly(0, z, a, f, chain=chain)
    want = ops[0].poly(z, a, psi)
    assert rel(lat.spinor_numpy(out), want) < 1e-12
    v = a * psi
    for k in range(6):
        assert rel(lat.spinor_numpy(chain[k]), v) < 1e-12
        v = ops[0].K(v) - z[k] * v
    # no chain, conjugated roots in another order
    zc = [np.conj(r) for r in z[::-1]]
    out2 = lat.apply_poly(1, zc, 1.0, f)
    assert rel(lat.spinor_numpy(out2), ops[1].poly(zc, 1.0, psi)) < 1e-12


def test_apply_poly_fp32_error(setup):
    """FP32 filter with its chain: error against the FP64 oracle stated, at the FP32
    rounding level of a degree-6 product."""
    from paper_1609_02652_amd import pfmp
    from paper_1609_02652_amd.pfmp import F32
    dims, U, lat, ops = setup
    z, a = pfmp.chebyshev(6, 1.2, 0.9)
    psi = synth.gaussian_spinor(lat.Vh, 21)
    f = lat.pack_spinor(psi, prec=F32)
    chain = [lat.field(prec=F32) for _ in range(6)]
    out = lat.apply_poly(0, z, a, f, chain=chain, prec=F32)
    e = rel(lat.spinor_numpy(out, prec=F32), ops[0].poly(z, a, psi))
    print("fp32 P(K) rel err", e)
    assert e < 1e-5
    v = a * psi
    for k in range(6):
        assert rel(lat.spinor_numpy(chain[k], prec=F32), v) < 1e-5
        v = ops[0].K(v) - z[k] * v
    # widening to FP64 is exact; narrowing rounds to nearest
    from paper_1609_02652_amd.pfmp import F64
    w = lat.convert_spinor(out, F32, F64)
    assert np.array_equal(lat.spinor_numpy(w), lat.spinor_numpy(out, prec=F32))
    n32 = lat.convert_spinor(lat.pack_spinor(psi), F64, F32)
    assert np.array_equal(lat.spinor_numpy(n32, prec=F32), psi.astype(np.complex64).astype(np.complex128))


@pytest.mark.parametrize("op", [0, 1])
def test_fermion_force(setup, op):
    dims, U, lat, ops = setup
    pairs_np = [(synth.gaussian_spinor(lat.Vh, 30 + k), synth.gaussian_spinor(lat.Vh, 40 + k), c)
                for k, c in enumerate([1.0, 0.3 - 0.7j, -2.0 + 0.1j])]
    F = lat.pack_momenta(np.zeros((lat.V, 4, 8)))
    lat.fermion_force(op, [(lat.pack_spinor(x), lat.pack_spinor(y), c) for x, y, c in pairs_np], F)
    got = lat.unpack_momenta(F).cpu().numpy()
    want = ops[op].force_bilinear(pairs_np)
    assert rel(got, want) < 1e-12


@pytest.mark.parametrize("op", [0, 1])
def test_fermion_force_fp32(setup, op):
    """FP32 spinor pairs (FORCE_F32: odd-site intermediates by the FP32 operator, the
    force summed in FP64) against the FP64 oracle on the same FP32-rounded vectors; nine
    pairs, so two launches of at most eight.  Error stated, at the FP32 rounding level."""
    from paper_1609_02652_amd.pfmp import F32, FORCE_F32
    dims, U, lat, ops = setup
    pairs_np = []
    for k in range(9):
        x = synth.gaussian_spinor(lat.Vh, 60 + k).astype(np.complex64).astype(np.complex128)
        y = synth.gaussian_spinor(lat.Vh, 70 + k).astype(np.complex64).astype(np.complex128)
        pairs_np.append((x, y, complex(np.cos(k), np.sin(0.7 * k))))
    F = lat.pack_momenta(np.zeros((lat.V, 4, 8)))
    lat.fermion_force(op, [(lat.pack_spinor(x, prec=F32), lat.pack_spinor(y, prec=F32), c)
                           for x, y, c in pairs_np], F, flags=FORCE_F32)
    got = lat.unpack_momenta(F).cpu().numpy()
    want = ops[op].force_bilinear(pairs_np)
    e = rel(got, want)
    print("fp32 fermion force rel err", e)
    assert e < 1e-5


def test_fermion_force_parts(setup):
    """Hop-only plus clover-only equals the full derivative."""
    from paper_1609_02652_amd.pfmp import FORCE_HOP, FORCE_CLOVER
    dims, U, lat, ops = setup
    x, y = synth.gaussian_spinor(lat.Vh, 50), synth.gaussian_spinor(lat.Vh, 51)
    fx, fy = lat.pack_spinor(x), lat.pack_spinor(y)
    Fa = lat.pack_momenta(np.zeros((lat.V, 4, 8)))
    lat.fermion_force(0, [(fx, fy, 1.0)], Fa, flags=FORCE_HOP)
    lat.fermion_force(0, [(fx, fy, 1.0)], Fa, flags=FORCE_CLOVER)
    Fb = lat.pack_momenta(np.zeros((lat.V, 4, 8)))
    lat.fermion_force(0, [(fx, fy, 1.0)], Fb)
    a, b = lat.unpack_momenta(Fa).cpu().numpy(), lat.unpack_momenta(Fb).cpu().numpy()
    assert rel(a, b) < 1e-13


def test_logdet_and_gauge_force(setup):
    dims, U, lat, ops = setup
    F = lat.pack_momenta(np.zeros((lat.V, 4, 8)))
    lat.logdet_force(0, F, coef=0.7)
    assert rel(lat.unpack_momenta(F).cpu().numpy(), ops[0].force_logdet(coef=0.7)) < 1e-12
    G = lat.pack_momenta(np.zeros((lat.V, 4, 8)))
    lat.gauge_force(5.7, G)
    assert rel(lat.unpack_momenta(G).cpu().numpy(), oracle.force_gauge(dims, U, 5.7)) < 1e-12


def test_actions(setup):
    dims, U, lat, ops = setup
    assert abs(lat.gauge_action(5.6) - oracle.gauge_action(dims, U, 5.6)) < 1e-12 * oracle.gauge_action(dims, U, 5.6)
    P = synth.gaussian_momenta(lat.V, 7)
    assert abs(lat.kinetic(lat.pack_momenta(P)) - oracle.kinetic(P)) < 1e-12 * oracle.kinetic(P)


def test_update_gauge_and_momenta(setup):
    from paper_1609_02652_amd.pfmp import Lattice
    dims, U, _, _ = setup
    lat = Lattice(dims)
    lat.set_gauge(U)
    lat.set_operator(0, 0.124, 1.25)
    P = synth.gaussian_momenta(lat.V, 8)
    Pd = lat.pack_momenta(P)
    lat.update_gauge(0.37, Pd)
    Uo = U.copy()
    oracle.update_gauge(dims, 0.37, P, Uo)
    Ug = lat.get_gauge().cpu().numpy()
    assert np.max(np.abs(Ug - Uo)) < 1e-14
    # the clover field was rebuilt on the new links
    o2 = oracle.Operator(dims, Uo, 0.124, 1.25)
    assert abs(lat.logdet_action(0) - o2.logdet_action()) < 1e-12 * abs(o2.logdet_action())
    F = synth.gaussian_momenta(lat.V, 9)
    lat.update_momenta(0.25, lat.pack_momenta(F), Pd)
    assert np.max(np.abs(lat.unpack_momenta(Pd).cpu().numpy() - (P - 0.25 * F))) < 1e-15
    lat.close()


def test_force_at_bench_shape_sampled():
    """16^3 x 32, the solve-benchmark lattice: the force on sampled links against
    the oracle evaluated link by link."""
    from paper_1609_02652_amd.pfmp import Lattice
    dims = (16, 16, 16, 32)
    U = synth.random_gauge(dims, seed=11)
    lat = Lattice(dims)
    lat.set_gauge(U)
    lat.set_operator(0, 0.1340, 1.6)
    x, y = synth.gaussian_spinor(lat.Vh, 60), synth.gaussian_spinor(lat.Vh, 61)
    F = lat.pack_momenta(np.zeros((lat.V, 4, 8)))
    lat.fermion_force(0, [(lat.pack_spinor(x), lat.pack_spinor(y), 0.5 + 0.5j)], F)
    lat.logdet_force(0, F)
    got = lat.unpack_momenta(F).cpu().numpy().reshape(-1, 8)
    rng = np.random.default_rng(0)
    links = np.sort(rng.choice(lat.V * 4, 64, replace=False))
    op = oracle.Operator(dims, U, 0.1340, 1.6)
    want = op.force_bilinear([(x, y, 0.5 + 0.5j)], links=links)
    op.force_logdet(want, links=links)
    want = want.reshape(-1, 8)[links]
    assert rel(got[links], want) < 1e-12
    lat.close()
