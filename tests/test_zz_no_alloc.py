"""The allocation-free Khat entry point (static device scratch) against pfmp_apply_MdagM,
through the C-ABI: two calls in a row on one GPU, the second on a smaller lattice, each
bit for bit equal to the allocating entry point (same kernels), in FP64 and FP32; a
lattice beyond the scratch limit is refused."""
import numpy as np
import pytest
import torch

from paper_1609_02652_amd import synth

pytestmark = pytest.mark.gpu


def _check(dims, seed, prec):
    from paper_1609_02652_amd.pfmp import Lattice
    print("case", dims, "prec", prec, flush=True)
    lat = Lattice(dims)
    try:
        lat.set_gauge(synth.random_gauge(dims, seed=seed))
        lat.set_operator(0, 0.1340, 1.6)
        x = lat.pack_spinor(synth.gaussian_spinor(lat.Vh, seed + 1), prec=prec)
        want = lat.apply_MdagM(0, x, prec=prec)
        out = lat.field(prec=prec)
        got = lat.apply_MdagM_noalloc(0, x, out, prec=prec)
        assert torch.equal(got, want)
    finally:
        lat.close()


@pytest.mark.parametrize("prec_name", ["f64", "f32"])
def test_noalloc_khat_matches_allocating(prec_name):
    from paper_1609_02652_amd.pfmp import F64, F32
    prec = F64 if prec_name == "f64" else F32
    _check((16, 16, 16, 32), 3, prec)     # first call on this GPU's scratch
    _check((6, 4, 4, 8), 4, prec)         # a second, smaller one reusing it


def test_noalloc_refuses_lattice_beyond_limit():
    from paper_1609_02652_amd.pfmp import Lattice, PfmpError, F64
    dims = (32, 32, 32, 64)               # two FP64 fields of 201 MB each exceed 128 MiB
    lat = Lattice(dims)
    try:
        x = lat.field()
        with pytest.raises(PfmpError) as e:
            lat.apply_MdagM_noalloc(0, x, lat.field(), prec=F64)
        assert e.value.code == -1
    finally:
        lat.close()
