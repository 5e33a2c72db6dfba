"""Host-side logic of the benchmark (no GPU): the one-GPU refusal, the traffic record that
the roofline line reads, and the CG iteration byte counts it prices the solves at."""
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def _record():
    text = open(os.path.join(ROOT, "profiles", "hop_fp64_pmc_traffic.md")).read()
    return json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))


def test_traffic_record_is_consistent():
    """The recorded traffic is FETCH x factor + WRITE of the table, and the ratios stated
    against the algorithmic and moved bytes follow from the recorded numbers."""
    rec = _record()
    for f in rec["sources"]:
        assert os.path.exists(os.path.join(ROOT, f)), f
    t = rec["traffic_bytes_per_launch"]["32x32x32x64"]
    algo = rec["algorithmic_bytes_per_launch"]["32x32x32x64"]
    moved = rec["moved_bytes_per_launch"]["32x32x32x64"]
    # 1,048,576 output sites at 32^3 x 64: 1,536 B algorithmic and 1,152 B moved per site
    assert algo == 1048576 * 1536 and moved == 1048576 * 1152
    text = open(os.path.join(ROOT, "profiles", "hop_fp64_pmc_traffic.md")).read()
    fetch = float(re.search(r"plain hop, FP64, CLOV=0 LM=3 \| 32\^3x64 \(2097152\) \| \d+ \| ([\d.]+) \| ([\d.]+)",
                            text).group(1))
    write = float(re.search(r"plain hop, FP64, CLOV=0 LM=3 \| 32\^3x64 \(2097152\) \| \d+ \| ([\d.]+) \| ([\d.]+)",
                            text).group(2))
    assert abs((fetch * rec["fetch_factor"] + write * rec["write_factor"]) * 1024 - t) / t < 1e-4


def test_traffic_reported_only_for_the_recorded_sources(tmp_path, monkeypatch):
    """pmc_traffic gives the recorded bytes while the kernel sources hash to the recorded
    value and None once any of them differs."""
    rec = _record()
    assert bench.pmc_traffic("32x32x32x64") == rec["traffic_bytes_per_launch"]["32x32x32x64"]
    assert bench.pmc_traffic("16x16x16x32") is None
    # a copy of the tree's sources with one byte changed
    fake = tmp_path / "root"
    for f in rec["sources"] + ["profiles/hop_fp64_pmc_traffic.md"]:
        dst = fake / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_bytes(open(os.path.join(ROOT, f), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(fake))
    assert bench.pmc_traffic("32x32x32x64") == rec["traffic_bytes_per_launch"]["32x32x32x64"]
    p = fake / rec["sources"][0]
    p.write_bytes(p.read_bytes() + b"\n")
    assert bench.pmc_traffic("32x32x32x64") is None


@pytest.mark.parametrize("prec,real_bytes", [("f64", 8), ("f32", 4)])
def test_cg_iteration_bytes(prec, real_bytes):
    """Per even site: two stage-1 launches (links 8 x 18, spinor in, clover 72, out), stage 2
    (links, T, p, clover, out), stage 4 (links, T', t, clover, p, x and r read and written) and
    the p update (r, p read and written): 1 272 reals."""
    links, spinor, clover = 8 * 18, 24, 72
    stage1 = links + spinor + clover + spinor
    stage2 = links + 2 * spinor + clover + spinor
    stage4 = links + 3 * spinor + clover + 4 * spinor
    update = 3 * spinor
    assert bench.CG_ITER_BYTES[prec] == real_bytes * (2 * stage1 + stage2 + stage4 + update)


def test_light_quark_spec():
    """The light-quark workload's action: the filter nest (6, 20, 62) on the 0.120 slot, its
    correction with the first ratio on one scale, the lightest ratio on a scale of its own,
    S_det of the 0.1370 slot, and the tolerance passed through."""
    from paper_1609_02652_amd.pfmp import Lattice, TERM_KINDS

    class Stub:
        spec = staticmethod(Lattice.spec)

    sp = bench.config5_spec(Stub(), (32, 8, 4, 16, 48), tol=1e-12, tau=0.5)
    kinds = {v: k for k, v in TERM_KINDS.items()}
    got = [(kinds[sp.terms[j].kind], sp.terms[j].op, sp.terms[j].op2, sp.terms[j].n, sp.terms[j].n1,
            sp.terms[j].steps) for j in range(sp.nterms)]
    assert got == [("poly", 1, -1, 6, 0, 8), ("polyq", 1, -1, 20, 6, 8), ("polyq", 1, -1, 62, 20, 8),
                   ("polycorr", 1, -1, 62, 0, 4), ("ratio", 1, 2, 0, 0, 4), ("ratio", 2, 3, 0, 0, 16),
                   ("ratio", 3, 0, 0, 0, 48)]
    assert (sp.gauge_steps, sp.det_op, sp.tol, sp.tau, sp.beta) == (32, 0, 1e-12, 0.5, bench.C5_BETA)
    assert bench.C5_HASEN == (0.120, 0.130, 0.135) and bench.C5_KAPPA == 0.1370
    # (p1 + 1) | (p2 + 1) for every level of the nest (App. A factorisation)
    p = bench.C5_NEST
    assert all((p[k + 1] + 1) % (p[k] + 1) == 0 for k in range(len(p) - 1))
