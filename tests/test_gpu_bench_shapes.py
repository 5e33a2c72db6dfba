"""GPU parity at the benchmark's full lattice sizes, 16^3 x 32 (the solve and
trajectory lattice) and 32^3 x 64 (the bandwidth lattice), in the launch
configuration the benchmark times: the visit order and link-load mode chosen by
the autotuner.  The FP64 hop D_oe, Mhat and Mhat^dag are compared on sampled
output sites with the oracle evaluated site by site; the FP32 and FP16-storage Mhat
errors against the same samples are stated."""
import numpy as np
import pytest

import oracle
from paper_1609_02652_amd import synth

pytestmark = pytest.mark.gpu

KAPPA, CSW = 0.1340, 1.6


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.mark.parametrize("dims", [(16, 16, 16, 32), (32, 32, 32, 64)], ids=lambda d: "x".join(map(str, d)))
def test_operator_sampled_at_bench_shape(dims):
    from paper_1609_02652_amd.pfmp import Lattice, F32, F16
    print("case", dims, flush=True)
    U = synth.random_gauge(dims, seed=5)
    lat = Lattice(dims)
    try:
        lat.set_gauge(U)
        lat.set_operator(0, KAPPA, CSW)
        tune = lat.autotune(0)
        print("tuning", tune, "links rebuilt", lat.link_reconstruct(), flush=True)
        psi = synth.gaussian_spinor(lat.Vh, 1)
        x = lat.pack_spinor(psi)
        rng = np.random.default_rng(2)
        sites = np.unique(np.concatenate([[0, lat.Vh - 1], rng.choice(lat.Vh, 254, replace=False)]))
        hop = lat.spinor_numpy(lat.apply_hop(1, x))[sites]
        assert rel(hop, oracle.sample_sites(dims, U, KAPPA, CSW, psi, sites, "hop")) < 1e-12
        want = {}
        for dag in (False, True):
            want[dag] = oracle.sample_sites(dims, U, KAPPA, CSW, psi, sites, "M", dagger=dag)
            got = lat.spinor_numpy(lat.apply_M(0, x, dagger=dag))[sites]
            assert rel(got, want[dag]) < 1e-12
        x32 = lat.pack_spinor(psi, prec=F32)
        e32 = rel(lat.spinor_numpy(lat.apply_M(0, x32, prec=F32), prec=F32)[sites], want[False])
        print("fp32 Mhat rel err on the samples", e32, flush=True)
        assert e32 < 2e-6
        # FP16 spinor storage (input rounded, the odd intermediate and the result stored in
        # FP16 with a per-site scale) with the FP16 and with the FP32 copies of links and clover
        for half_links in (1, 0):
            lat.half_links(half_links)
            e16 = rel(lat.spinor_numpy(lat.apply_M(0, x32, prec=F16), prec=F32)[sites], want[False])
            print("fp16-storage Mhat rel err on the samples (half links %d): %.3e" % (half_links, e16), flush=True)
            assert e16 < 3e-3
        lat.half_links(1)
    finally:
        lat.close()


def test_operator_sampled_at_light_quark_shape():
    """The light-quark trajectory lattice, 48^3 x 96 at kappa 0.1370, c_sw 1.6 (its lightest
    operator), on the seeded start field: the FP64 Mhat and Mhat^dag in the launch
    configuration the autotuner picks, against the oracle on sampled output sites."""
    from paper_1609_02652_amd.pfmp import Lattice
    dims, kappa = (48, 48, 48, 96), 0.1370
    print("case", dims, kappa, flush=True)
    U = synth.random_gauge(dims, seed=0)
    lat = Lattice(dims)
    try:
        lat.set_gauge(U)
        lat.set_operator(0, kappa, CSW)
        print("tuning", lat.autotune(0), "links rebuilt", lat.link_reconstruct(), flush=True)
        psi = synth.gaussian_spinor(lat.Vh, 1)
        x = lat.pack_spinor(psi)
        rng = np.random.default_rng(4)
        sites = np.unique(np.concatenate([[0, lat.Vh - 1], rng.choice(lat.Vh, 126, replace=False)]))
        for dag in (False, True):
            got = lat.spinor_numpy(lat.apply_M(0, x, dagger=dag))[sites]
            e = rel(got, oracle.sample_sites(dims, U, kappa, CSW, psi, sites, "M", dagger=dag))
            print("Mhat%s rel err on the samples: %.3e" % ("^dag" if dag else "", e), flush=True)
            assert e < 1e-12
    finally:
        lat.close()
