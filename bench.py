"""Benchmark of the PF-MP HMC hot path on one MI355X.

One step = one PF-MP HMC trajectory (paper eq. pfmp_action, App. B integrator,
App. C forces) on the 16^3 x 32 clover workload: links from quenched HMC at
beta 5.7 from the seeded start, kappa 0.1340, c_sw 1.6, Hasenbusch kappa' 0.1300,
degree-4 Chebyshev filter (mu, nu) = (1.2, 0.9).  The filter / correction / gauge
step counts (120, 20, 480) are those of the paper's best PF-MP run; the ratio term
takes 20 steps (6 in the paper, whose ensemble and masses differ) and S_det, which
the paper's Wilson runs do not have, 120.  tau = 1, every solve to relative
residual 1e-10.  Inputs are seeded synthetic fields already resident in HBM when
the timed region starts.

The JSON line also reports the CG solve time at 1e-10 on the same lattice, the
hopping-kernel bandwidth measured with HIP events on the library's stream (the
roofline of the dominant kernel), and the FP64 oracle timed on the host cores on a
bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DIMS = (16, 16, 16, 32)
KAPPA, KAPPA_H, CSW, BETA = 0.1340, 0.1300, 1.6, 5.7
STEPS = dict(ratio=20, corr=20, poly=120, gauge=480, det=120)
TOL = 1e-10


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_lattice(dims, U):
    from paper_1609_02652_amd.pfmp import Lattice
    lat = Lattice(dims)
    lat.set_gauge(U)
    lat.set_operator(0, KAPPA, CSW)
    lat.set_operator(1, KAPPA_H, CSW)
    return lat


def pfmp_spec(lat, steps=STEPS, tol=TOL, **kw):
    terms = [dict(kind="poly", op=1, n=4, mu=1.2, nu=0.9, steps=steps["poly"]),
             dict(kind="polycorr", op=1, n=4, mu=1.2, nu=0.9, steps=steps["corr"]),
             dict(kind="ratio", op=1, op2=0, steps=steps["ratio"])]
    return lat.spec(BETA, terms, steps["gauge"], det_op=0, tol=tol, det_steps=steps["det"], **kw)


def time_kernel(lat, fn, reps):
    """Average duration of fn() (one kernel launch) from HIP events on the library's stream."""
    import torch
    s = lat.stream
    for _ in range(3):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


BATCH_LAYOUTS = ((1, "multi"), (2, "multi2"), (0, "wg"))


def batch_apply(lat, reps=20, layouts=BATCH_LAYOUTS):
    """4-RHS Khat against 4 single-RHS Khat in FP64 and FP32, for 4 sources of one operator and
    for the Hasenbusch chain's operators (kappa 0.1340, 0.1300, 0.1250, 0.1340), in the
    multi-rhs layout (each link load shared by the rhs of a lane pair: the default group of 4,
    and groups of 2) and in the workgroup-per-rhs layout: time per right-hand side relative to
    a single one."""
    from paper_1609_02652_amd import synth
    from paper_1609_02652_amd.pfmp import F64, F32
    lat.set_operator(2, 0.1250, CSW)
    res = {}
    for pname, prec in (("f64", F64), ("f32", F32)):
        xs = [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 40 + k), prec=prec) for k in range(4)]
        outs = [lat.field(prec=prec) for _ in range(4)]
        t1 = time_kernel(lat, lambda: lat.apply_MdagM(0, xs[0], out=outs[0], prec=prec), reps)
        for oname, ops in (("same_op", [0, 0, 0, 0]), ("chain", [0, 1, 2, 0])):
            for multi, lname in layouts:
                lat.batch_layout(multi)
                t4 = time_kernel(lat, lambda: lat.apply_MdagM_batch(ops, xs, outs, prec=prec), reps)
                res["%s_%s_%s" % (pname, oname, lname)] = {
                    "single_K_us": round(t1 * 1e6, 1), "batch_K_us": round(t4 * 1e6, 1),
                    "per_rhs_vs_single": round(t4 / 4 / t1, 3)}
        lat.batch_layout(True)
    return res


def hop_roofline(dims, U, reps=200, extra=None):
    """The plain FP64 hop D_oe and Mhat after autotuning, timed with HIP events on the
    library stream.  bytes_hop counts the bytes the hop kernel must move per output
    site: 8 links (12 reals each when the third row is rebuilt, else 18) plus the
    input and output spinors (24 reals each); bytes_M adds the second hop, the two
    clover applies (72 reals each) and the axpy input."""
    from paper_1609_02652_amd.pfmp import F64
    lat = make_lattice(dims, U)
    tune = lat.autotune(0)
    from paper_1609_02652_amd import synth
    x = lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 1))
    out = lat.field()
    # apply_M = stage 1 (hop + A^-1) then stage 2 (hop + A_ee + axpy); time the pair
    # and the plain hop separately
    t_plain = time_kernel(lat, lambda: lat.apply_hop(1, x, out=out), reps)
    t_m = time_kernel(lat, lambda: lat.apply_M(0, x, out=out, prec=F64), reps)
    # links are SU(3): the kernels read 2 of the 3 rows (12 reals per link)
    link_reals = 12 if lat.link_reconstruct() else 18
    bytes_plain = lat.Vh * (8 * link_reals + 24 + 24) * 8
    bytes_m = lat.Vh * (2 * (8 * link_reals + 24 + 24) + 72 * 2 + 24) * 8
    more = extra(lat) if extra else None
    lat.close()
    return {"t_hop": t_plain, "bytes_hop": bytes_plain, "t_M": t_m, "bytes_M": bytes_m, "Vh": lat.Vh,
            "link_reals": link_reals, "tune": tune, "extra": more}


def pmc_traffic(lattice):
    """HBM bytes per launch of the plain FP64 hop from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (scaled by the counters' reading for a copy of
    known size), or None when the kernel sources have changed since they were
    taken."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, "profiles", "hop_fp64_pmc_traffic.md")).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None
        return rec["traffic_bytes_per_launch"].get(lattice)
    except (OSError, ValueError, KeyError, AttributeError):
        return None


def roofline_only(reps):
    """Only the hopping kernels (16^3x32 and 32^3x64) and a plain copy of known size,
    for hardware-counter runs: FETCH_SIZE / WRITE_SIZE of the copy calibrate the
    counters of the hopping kernel."""
    import torch
    from paper_1609_02652_amd import synth
    from paper_1609_02652_amd.pfmp import F32, F16
    out = {}

    def lowprec(lt):
        # Khat with FP32 fields and with FP16 storage (the mixed solvers' stage kernels)
        x32 = lt.pack_spinor(synth.gaussian_spinor(lt.Vh, 1), prec=F32)
        o32 = lt.field(prec=F32)
        return {"Khat_f32_us": round(time_kernel(lt, lambda: lt.apply_MdagM(0, x32, out=o32, prec=F32), reps) * 1e6, 2),
                "Khat_f16_us": round(time_kernel(lt, lambda: lt.apply_MdagM(0, x32, out=o32, prec=F16), reps) * 1e6, 2)}

    for dims in (DIMS, (32, 32, 32, 64)):
        r = hop_roofline(dims, synth.random_gauge(dims, seed=5), reps=reps, extra=lowprec)
        out["x".join(map(str, dims))] = dict({"hop_us": round(r["t_hop"] * 1e6, 2), "tuning": r["tune"],
                                              "hop_GBps": round(r["bytes_hop"] / r["t_hop"] / 1e9, 1),
                                              "hop_bytes": r["bytes_hop"], "Mhat_us": round(r["t_M"] * 1e6, 2)},
                                             **r["extra"])
    n = 256 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    out["copy_256MiB"] = {"us": round(t * 1e6, 2), "GBps_read_plus_write": round(2 * n * 8 / t / 1e9, 1)}
    print(json.dumps(out), flush=True)


def batch_only(reps, zts=None):
    """Only the multi-RHS Khat comparison at 32^3x64 (after autotuning) and a plain copy of
    known size, for hardware-counter runs on the batched stencils.  zts: also repeat the
    comparison (groups of 4 rhs per lane pair) under each of these site visit orders."""
    from paper_1609_02652_amd import synth
    big = (32, 32, 32, 64)
    lat = make_lattice(big, synth.random_gauge(big, seed=5))
    out = {"tuning": lat.autotune(0)}
    out["multi_rhs_Khat_32x32x32x64"] = batch_apply(lat, reps)
    for zt in zts or ():
        lat.site_order(zt)
        out["site_order_zt%d" % zt] = r = batch_apply(lat, reps, layouts=BATCH_LAYOUTS[:1])
        log("zt %d: %s" % (zt, r))
    lat.close()
    out["copy_256MiB"] = copy_bandwidth(reps)
    print(json.dumps(out), flush=True)


def copy_bandwidth(reps=20):
    """Device-to-device copy of 256 MiB (read + write bytes per second), for context."""
    import torch
    n = 256 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    return {"bytes": 2 * n * 8, "us": round(t * 1e6, 2), "GBps": round(2 * n * 8 / t / 1e9, 1)}


def host_info():
    """CPU model and logical core count of the host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def oracle_cg_solve(threads=None):
    """The oracle (plain C, FP64) solving one source of the solve workload: Khat (kappa 0.1340,
    c_sw 1.6) on the seeded 16^3 x 32 start field, CG to 1e-10 from x = 0.  The oracle never sees
    the GPU's thermalised field, so it solves on the seeded start field (the cost of an iteration
    does not depend on the link values; the iteration count is stated).  threads: OpenMP threads
    (the environment's default when None)."""
    import oracle
    from paper_1609_02652_amd import synth
    U = synth.random_gauge(DIMS, seed=0)
    t0 = time.perf_counter()
    op = oracle.Operator(DIMS, U, KAPPA, CSW)
    t_setup = time.perf_counter() - t0
    b = synth.gaussian_spinor(op.Vh, 1)
    t0 = time.perf_counter()
    x, info = op.cg(b, tol=TOL)
    t = time.perf_counter() - t0
    res = float(np.linalg.norm(op.K(x) - b) / np.linalg.norm(b))
    return {"s": round(t, 3), "setup_s": round(t_setup, 3), "iters": info["iters"], "true_res": res}


def oracle_config1_trajectory():
    """The correctness workload's trajectory on the oracle (4^4, kappa 0.120 / 0.110, c_sw
    1.0, degree-4 filter, 2MN steps (10, 20, 40, 80), CG 1e-12), seconds."""
    from oracle import hmc
    from paper_1609_02652_amd import synth
    dims = (4, 4, 4, 4)
    U0 = synth.random_gauge(dims, seed=0)
    terms = [dict(kind="poly", kappa=0.110, n=4, mu=1.2, nu=0.9, steps=40),
             dict(kind="polycorr", kappa=0.110, n=4, mu=1.2, nu=0.9, steps=20),
             dict(kind="ratio", kappa_num=0.110, kappa_den=0.120, steps=10)]
    spec = dict(dims=dims, beta=5.6, csw=1.0, kappa=0.120, gauge_steps=80, terms=terms)
    P0 = synth.gaussian_momenta(256, 100)
    etas = [synth.gaussian_spinor(128, 20 + j) for j in range(3)]
    t0 = time.perf_counter()
    ref = hmc.trajectory(spec, U0, P0, etas, u=float(synth.uniform(200)[0]), tol=1e-12)
    return {"s": round(time.perf_counter() - t0, 3), "dH": ref["dH"], "accept": bool(ref["accept"])}


def cpu_full(args):
    """The oracle on the host: one full CG solve of the solve workload (16^3 x 32, 1e-10) and
    the full correctness-workload trajectory (4^4), each in a child process with 1 OpenMP
    thread and with all host threads."""
    import subprocess
    out = dict(host_info())
    counts = [1, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))]
    for what in ("cg", "traj"):
        for n in counts:
            env = dict(os.environ, OMP_NUM_THREADS=str(n))
            log("oracle %s with %d thread(s)" % (what, n))
            r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-child", what], env=env,
                               capture_output=True, text=True, check=True)
            out["%s_threads_%d" % (what, n)] = json.loads(r.stdout.strip().splitlines()[-1])
            log("  %s" % out["%s_threads_%d" % (what, n)])
    print(json.dumps({"cpu_full": out}), flush=True)


def cpu_baseline():
    """The oracle on the host cores: one full CG solve of the solve workload (16^3 x 32,
    kappa 0.1340, 1e-10) with the host's OpenMP threads, in the headline's unit (s per solve)."""
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    r = oracle_cg_solve()
    return dict({"value": r["s"], "unit": "s/solve", "cores": threads, "kind": "oracle",
                 "sample": "one full CG solve to 1e-10 (source 1, seeded 16^3x32 start field, %s iterations, "
                           "true residual %.1e; clover set-up %.1f s excluded)" % (r["iters"], r["true_res"],
                                                                                  r["setup_s"])},
                **host_info())


def thermalise(lat, ntraj, gauge_steps=128, beta=BETA):
    """Quenched HMC (Wilson gauge action at beta, 2MN, tau = 1) from the seeded start:
    the links the solver and trajectory benchmarks run on."""
    from paper_1609_02652_amd import synth
    sp = lat.spec(beta, [], gauge_steps, det_op=-1)
    acc = 0
    for k in range(ntraj):
        st = lat.trajectory(sp, lat.pack_momenta(synth.gaussian_momenta(lat.V, 7000 + k)), [],
                            synth.uniform(8000 + k)[0])
        acc += st["accept"]
    plaq = 1.0 - lat.gauge_action(beta) / (beta * 6 * lat.V)
    log("quenched thermalisation: %d trajectories, acceptance %.2f, plaquette %.5f" % (ntraj, acc / max(ntraj, 1),
                                                                                      plaq))
    return {"trajectories": ntraj, "accept_rate": acc / max(ntraj, 1), "plaquette": round(plaq, 6)}


def cg_bench(lat, nsrc, warmup=1):
    """The solve workload: CG on Khat (kappa 0.1340) to 1e-10, one Gaussian source at a time,
    in FP64, FP32 + FP64 reliable updates, and FP32 arithmetic with FP16 storage + FP64
    reliable updates.  Per precision: `warmup` untimed solves, then exactly nsrc solves timed
    together between two device synchronisations (mean seconds per solve); also the median
    per solve, iterations, the worst FP64 true residual and the worst ||x - x_FP64|| / ||x_FP64||
    over the same sources (FP64 solutions kept from the FP64 pass, compared outside the
    timing)."""
    import torch
    from paper_1609_02652_amd import synth
    from paper_1609_02652_amd.pfmp import F64, F32, F16
    res = {}
    srcs = [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 1 + s)) for s in range(nsrc)]
    xs = [lat.field() for _ in range(nsrc)]
    x64 = []
    for name, prec in (("f64", F64), ("f32", F32), ("f16", F16)):
        for w in range(warmup):
            lat.cg_solve(0, srcs[w % nsrc], x=xs[0], tol=TOL, prec=prec)
        sts, per = [], []
        torch.cuda.synchronize()
        t_all = time.perf_counter()
        for k in range(nsrc):
            t0 = time.perf_counter()
            _, st = lat.cg_solve(0, srcs[k], x=xs[k], tol=TOL, prec=prec)
            per.append(time.perf_counter() - t0)   # each solve ends on a host read of its residual
            sts.append(st)
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t_all
        if prec == F64:
            x64 = [x.clone() for x in xs]
            errs = [0.0] * nsrc
        else:
            errs = [float(torch.linalg.vector_norm(x - y) / torch.linalg.vector_norm(y)) for x, y in zip(xs, x64)]
        res[name] = {"mean_s": round(t_all / nsrc, 6), "median_s": round(float(np.median(per)), 6),
                     "iters": int(np.median([st["iters"] for st in sts])),
                     "reliable_updates": int(np.median([st["reliable_updates"] for st in sts])),
                     "max_true_res": float(max(st["true_res"] for st in sts)),
                     "max_rel_err_vs_f64": float(max(errs))}
        log("cg %s: %s" % (name, res[name]))
    return res


def cg_iteration_roofline(lat, Vh, reps=2):
    """Per-iteration time of one CG solve (kappa 0.1340, 1e-10) in each precision on this
    lattice, priced at CG_ITER_BYTES per even site against the 8 TB/s peak."""
    import torch
    from paper_1609_02652_amd import synth
    from paper_1609_02652_amd.pfmp import F64, F32, F16
    b = lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 1))
    x = lat.field()
    out = {}
    for name, prec in (("f64", F64), ("f32", F32), ("f16", F16)):
        lat.cg_solve(0, b, x=x, tol=TOL, prec=prec)
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = lat.cg_solve(0, b, x=x, tol=TOL, prec=prec)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / st["iters"]
            best = t if best is None or t < best else best
        gbs = CG_ITER_BYTES[name] * Vh / best / 1e9
        out[name] = {"us_per_iter": round(best * 1e6, 1), "iters": st["iters"],
                     "bytes_per_iter_site": CG_ITER_BYTES[name], "GBps": round(gbs, 1),
                     "frac": round(gbs / HBM_PEAK_GBS, 3)}
        log("cg iteration %s: %s" % (name, out[name]))
    return out


# Algorithmic bytes of one CG iteration per even site, from the I/O of its five kernels (each
# input field counted once per site): stage 1 (hop + A_oo^-1): links 8 x 18, in 24, clover 72,
# out 24 reals; stage 2 (hop + A_ee + axpy, |t|^2): links, T 24, p 24, clover, out 24; stage 3
# as stage 1; stage 4 (hop + A_ee, x and r updates, |r|^2): links, T' 24, t 24, clover, p 24,
# x and r read and written 4 x 24; p update: r 24, p read and written 48.  FP64: 1272 reals
# x 8 B; FP32: x 4 B; FP16 storage: links and clover in binary16, the p / t / T fields as
# binary16 with a 4 B site scale, x and r in FP32.
CG_ITER_BYTES = {
    "f64": 8 * (264 + 288 + 264 + 384 + 72),
    "f32": 4 * (264 + 288 + 264 + 384 + 72),
    "f16": (144 * 2 + 52 + 72 * 2 + 52) * 2 + (144 * 2 + 52 + 52 + 72 * 2 + 52)
           + (144 * 2 + 52 + 52 + 72 * 2 + 52 + 4 * 96) + (96 + 2 * 52),
}


def cg_roofline(cg, Vh):
    """Achieved algorithmic bandwidth of each solve (iterations x CG_ITER_BYTES x Vh / time)
    as a fraction of the 8 TB/s HBM peak; at 16^3 x 32 the working set sits in the 256 MB
    last-level cache, so the fraction is against HBM, not the cache."""
    out = {}
    for k in ("f64", "f32", "f16"):
        b = cg[k]["iters"] * CG_ITER_BYTES[k] * Vh
        out[k] = {"bytes_per_iter_site": CG_ITER_BYTES[k], "GBps": round(b / cg[k]["median_s"] / 1e9, 1),
                  "frac": round(b / cg[k]["median_s"] / 1e9 / HBM_PEAK_GBS, 3),
                  "note": "16^3x32: the working set stays in the 256 MB last-level cache"}
    return out


def batch_bench(lat, reps=3):
    """Multi-RHS CG: the three solves of a Hasenbusch chain at one gauge field
    (kappa 0.1340, 0.1300, 0.1250 on slots 0, 1, 2) in one batched solve against the
    same three solves one after the other (FP64, 1e-10)."""
    import torch
    from paper_1609_02652_amd import synth
    ops = [0, 1, 2]
    bs = [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 700 + k)) for k in range(3)]
    xs = [lat.field() for _ in ops]
    lat.cg_solve_batch(ops, bs, xs=xs, tol=TOL)   # warm-up
    t_b, t_s = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, sts = lat.cg_solve_batch(ops, bs, xs=xs, tol=TOL)
        torch.cuda.synchronize()
        t_b.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        its = []
        for op, b, x in zip(ops, bs, xs):
            _, st = lat.cg_solve(op, b, x=x, tol=TOL)
            its.append(st["iters"])
        torch.cuda.synchronize()
        t_s.append(time.perf_counter() - t0)
    out = {"nrhs": 3, "kappas": [KAPPA, KAPPA_H, 0.1250], "batched_s": round(float(np.median(t_b)), 5),
           "sequential_s": round(float(np.median(t_s)), 5), "iters": [s["iters"] for s in sts],
           "max_true_res": float(max(s["true_res"] for s in sts)),
           "speedup": round(float(np.median(t_s)) / float(np.median(t_b)), 3)}
    log("batched solves: %s" % out)
    return out


def batched_force_bench():
    """The Hasenbusch chain of the batched-force workload on 24^3 x 48 (kappa 0.1360,
    0.1300, 0.1200, c_sw 1.6; heavy term on 0.1200 and ratio terms 0.1200/0.1300 and
    0.1300/0.1360): one 2MN step of all three terms (three force evaluations, three CG
    solves each to 1e-10), with the solves of each evaluation as one multi-RHS batch
    against one after another, in FP64 and in the mixed-precision mode (single solves:
    FP16-storage CG with FP64 reliable updates; batches: FP32 batched passes inside FP64
    residuals).  Seeded start links (the timing does not need thermalised ones)."""
    import torch
    from paper_1609_02652_amd import synth
    from paper_1609_02652_amd.pfmp import Lattice
    dims = (24, 24, 24, 48)
    lat = Lattice(dims)
    try:
        lat.set_gauge(synth.random_gauge(dims, seed=0))
        for k, kap in enumerate((0.1360, 0.1300, 0.1200)):
            lat.set_operator(k, kap, CSW)
        tune = lat.autotune(0)
        terms = [dict(kind="heavy", op=2, steps=1), dict(kind="ratio", op=2, op2=1, steps=1),
                 dict(kind="ratio", op=1, op2=0, steps=1)]
        U0 = lat.get_gauge().clone()
        phis = [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 800 + j)) for j in range(3)]
        out = {"lattice": "x".join(map(str, dims)), "nrhs": 3, "tuning": tune}
        from paper_1609_02652_amd.pfmp import F64, F16
        modes = {"f64_one_by_one": (F64, False), "f64_batched": (F64, True),
                 "mixed_one_by_one": (F16, False), "mixed_batched": (F16, True)}
        for name, (prec, batch) in list(modes.items()) * 2:   # the second pass of each is kept
            sp = lat.spec(5.8, terms, 1, det_op=-1, tau=0.02, batch=batch, solver_prec=prec)
            P = lat.pack_momenta(synth.gaussian_momenta(lat.V, 900))
            lat.set_gauge(U0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = lat.md_evolve(sp, P, phis)
            torch.cuda.synchronize()
            out[name] = {"s": round(time.perf_counter() - t0, 4), "solver_iters": st["solver_iters"]}
        out["batched_speedup_f64"] = round(out["f64_one_by_one"]["s"] / out["f64_batched"]["s"], 3)
        out["mixed_batched_vs_f64_one_by_one"] = round(out["f64_one_by_one"]["s"] / out["mixed_batched"]["s"], 3)
        lat.set_gauge(U0)
        return out
    finally:
        lat.close()


def learned_bench(lat, nsrc):
    """The learned preconditioner on Khat (kappa 0.1340): training vectors are
    residuals the solver itself produces (CG iterates 2, 6, 10, 14, 20, 30 of 4
    solves) plus 8 Gaussian vectors; Adam (300 full-batch steps) on the
    preconditioned-residual objective in the library's own forward / backward
    kernels; then flexible CG with the trained network on the benchmark sources to
    1e-10 (FP64 true residual), against plain FP64 CG on the same sources."""
    import torch
    from paper_1609_02652_amd import synth
    rs = []
    for s in range(4):
        b = lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 500 + s))
        _, pr = lat.cg_harvest(0, b, [2, 6, 10, 14, 20, 30], tol=1e-10)
        rs += [r for r, _ in pr]
    rs += [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 600 + k)) for k in range(8)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W, losses = lat.ptnet_train(synth.network_weights(4, scale=0.05), rs, steps=300, lr=1e-2, op=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    srcs = [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 1 + s)) for s in range(nsrc)]
    x = lat.field()
    lat.fcg_solve(0, W, srcs[0], x=x, tol=TOL)   # warm-up
    rows = []
    for b in srcs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = lat.fcg_solve(0, W, b, x=x, tol=TOL)
        torch.cuda.synchronize()
        rows.append((time.perf_counter() - t0, st["iters"], st["true_res"], st["reliable_updates"]))
    out = {"train_vectors": len(rs), "train_steps": 300, "train_s": round(t_train, 3),
           "loss_first": round(float(losses[0]), 4), "loss_last": round(float(losses[-1]), 4),
           "fcg_median_s": round(float(np.median([r[0] for r in rows])), 5),
           "fcg_iters": int(np.median([r[1] for r in rows])),
           "fallback_steps": int(max(r[3] for r in rows)),
           "max_true_res": float(max(r[2] for r in rows))}
    log("learned preconditioner: %s" % out)
    return out, W


def learned32_bench(args):
    """The learned preconditioner at the learning workload's size: 32^3 x 64, links from 10
    quenched HMC trajectories at beta = 5.9 (1024 2MN steps), clover kappa = 0.1365, c_sw = 1.6; training
    vectors from 4 CG solves (iterates 2, 6, 10, 14, 20, 30) and 8 Gaussian vectors, 150 Adam
    steps; then flexible CG with the trained network against plain FP64 CG and the
    FP32 and FP16-storage mixed CG (FP16 storage with the FP16 and with the FP32 copies of
    links and clover) on 3 sources, all to 1e-10."""
    import torch
    from paper_1609_02652_amd import synth
    from paper_1609_02652_amd.pfmp import F16, F32, Lattice
    dims = (32, 32, 32, 64)
    lat = Lattice(dims)
    lat.set_gauge(synth.random_gauge(dims, seed=0))
    therm = thermalise(lat, 10, gauge_steps=1024, beta=5.9)   # dH grows with the volume: finer steps than 16^3 x 32
    lat.set_operator(0, 0.1365, 1.6)
    log("autotune: %s" % lat.autotune(0))
    rs = []
    for s in range(4):
        b = lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 500 + s))
        _, pr = lat.cg_harvest(0, b, [2, 6, 10, 14, 20, 30], tol=1e-10)
        rs += [r for r, _ in pr]
    rs += [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 600 + k)) for k in range(8)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W, losses = lat.ptnet_train(synth.network_weights(4, scale=0.05), rs, steps=150, lr=1e-2, op=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    srcs = [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 1 + s)) for s in range(3)]
    x = lat.field()
    res = {}
    for name, fn in (("cg_f64", lambda b: lat.cg_solve(0, b, x=x, tol=TOL)),
                     ("cg_f32", lambda b: lat.cg_solve(0, b, x=x, tol=TOL, prec=F32)),
                     ("cg_f16", lambda b: lat.cg_solve(0, b, x=x, tol=TOL, prec=F16)),
                     ("cg_f16_fp32_links", lambda b: (lat.half_links(False),
                                                      lat.cg_solve(0, b, x=x, tol=TOL, prec=F16), lat.half_links(True))[1]),
                     ("fcg_learned", lambda b: lat.fcg_solve(0, W, b, x=x, tol=TOL))):
        fn(srcs[0])
        rows = []
        for b in srcs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = fn(b)
            torch.cuda.synchronize()
            rows.append((time.perf_counter() - t0, st["iters"], st["true_res"]))
        res[name] = {"median_s": round(float(np.median([r[0] for r in rows])), 4),
                     "iters": [r[1] for r in rows], "max_true_res": float(max(r[2] for r in rows))}
        log("learned32 %s: %s" % (name, res[name]))
    lat.close()
    print(json.dumps({"learned_32x32x32x64": dict(res, train_s=round(t_train, 2), train_vectors=len(rs),
                                                  loss=[round(float(losses[0]), 4), round(float(losses[-1]), 4)],
                                                  thermalisation=therm,
                                                  fcg_vs_cg_f64=round(res["cg_f64"]["median_s"] /
                                                                      res["fcg_learned"]["median_s"], 3))}),
          flush=True)


KAPPA_1 = 0.1250


def zoo_specs(lat, prec):
    """The paper's actions over the same terms (Sec. 2.2 eq. hasenbusch, 1poly, 2poly; Sec. 3
    PF-MP, 2MP, 1PF-2MP, 2PF-1MP) on the benchmark field: slots 0 = K (kappa 0.1340),
    1 = J (0.1300), 2 = J_1 (0.1250); degree-4 filters, the 2-filter actions with P_4
    inside P_24 (the paper's 2PF-1MP choice), gauge 480 and S_det 120 2MN steps, every
    solve to 1e-10.  Step counts are fixed, not tuned per action."""
    def p(kind, op, n, steps, n1=0):
        return dict(kind=kind, op=op, n=n, n1=n1, mu=1.2, nu=0.9, steps=steps)

    def r(op, op2, steps):
        return dict(kind="ratio", op=op, op2=op2, steps=steps)
    zoo = {
        "PF-MP": [p("poly", 1, 4, 120), p("polycorr", 1, 4, 20), r(1, 0, 20)],
        "1MP": [dict(kind="heavy", op=1, steps=120), r(1, 0, 20)],
        "2MP": [dict(kind="heavy", op=2, steps=120), r(2, 1, 40), r(1, 0, 20)],
        "1PF": [p("poly", 0, 4, 120), p("polycorr", 0, 4, 20)],
        "2PF": [p("poly", 0, 4, 120), p("polyq", 0, 24, 40, n1=4), p("polycorr", 0, 24, 20)],
        "2PF-1MP": [p("poly", 1, 4, 120), p("polyq", 1, 24, 40, n1=4), p("polycorr", 1, 24, 20), r(1, 0, 20)],
        "1PF-2MP": [p("poly", 2, 4, 120), p("polycorr", 2, 4, 20), r(2, 1, 20), r(1, 0, 20)],
    }
    return {k: lat.spec(BETA, v, STEPS["gauge"], det_op=0, tol=TOL, det_steps=STEPS["det"], solver_prec=prec)
            for k, v in zoo.items()}


def zoo_bench(args):
    """One timed trajectory (after one warm-up) of each action of zoo_specs, in plain FP64 and
    in the chosen mixed precision (FP16-storage CG), on the same inputs."""
    from paper_1609_02652_amd import synth
    from paper_1609_02652_amd.pfmp import F64, F16, Lattice
    lat = Lattice(DIMS)
    lat.set_gauge(synth.random_gauge(DIMS, seed=0))
    thermalise(lat, args.therm)
    for op, k in ((0, KAPPA), (1, KAPPA_H), (2, KAPPA_1)):
        lat.set_operator(op, k, CSW)
    log("autotune: %s" % lat.autotune(0))
    out = {}
    for mode, prec in (("f16", F16), ("f64", F64)):
        for name, sp in zoo_specs(lat, prec).items():
            t, sts = run_trajectories(lat, sp, 1, 1, 100)
            s = sts[0]
            out.setdefault(name, {})[mode] = {"s_per_traj": round(t, 4), "dH": round(s["dH"], 5),
                                              "kmults": s["kmults"], "solver_iters": s["solver_iters"],
                                              "nforce": s["nforce"]}
            log("zoo %s %s: %s" % (name, mode, out[name][mode]))
    lat.close()
    print(json.dumps({"zoo": out, "lattice": "x".join(map(str, DIMS)),
                      "kappas": {"K": KAPPA, "J": KAPPA_H, "J_1": KAPPA_1}}), flush=True)


def tune_bench(args):
    """The paper's tuning procedure (Sec. 2.4) for the PF-MP action on the benchmark field:
    maximal forces per row over 3 trajectories, steps with F_i h_i = const, the scale tuned
    to P_acc in [0.65, 0.75] (rounds of 8 trajectories), then the cost C = N_mat / P_acc with
    the tau_int-corrected error over a further 12 trajectories, in the chosen mixed
    precision."""
    from paper_1609_02652_amd import synth, tuner
    from paper_1609_02652_amd.pfmp import F16, Lattice
    lat = Lattice(DIMS)
    lat.set_gauge(synth.random_gauge(DIMS, seed=0))
    thermalise(lat, args.therm)
    lat.set_operator(0, KAPPA, CSW)
    lat.set_operator(1, KAPPA_H, CSW)
    log("autotune: %s" % lat.autotune(0))

    # S_det rides on the gauge scale here (its default): with a step count from its small
    # maximal force it becomes unstable at 2-3 steps, a stiffness the force size misses
    def build(steps):
        n_g, n_p, n_c, n_r = steps[:4]
        st = dict(poly=n_p, corr=n_c, ratio=n_r, gauge=n_g, det=0)
        return pfmp_spec(lat, steps=st, solver_prec=F16)
    start = [STEPS["gauge"], STEPS["poly"], STEPS["corr"], STEPS["ratio"]]
    T = tuner.StepTuner(lat, build, 3, seed=7000)
    t0 = time.perf_counter()
    F = T.measure_forces(start, 3)
    fmax = list(F[:4, 0])
    log("maximal forces (gauge, poly, corr, ratio, det): %s" % [round(f, 4) for f in fmax])
    c0 = fmax[3] / STEPS["ratio"]   # keep the ratio term's step at first
    hist, best = T.tune(fmax, c0)
    for c, steps, traj in hist:
        log("c %.5f steps %s dH %s" % (c, steps, [round(t[0], 4) for t in traj]))
    c, steps, _ = hist[best]
    chain = T.run(steps, 12)
    lat.close()
    dH = [t[0] for t in chain]
    acc = [t[1] for t in chain]
    nmat = [t[2] for t in chain]
    C, dC = tuner.cost(nmat, acc)
    print(json.dumps({"tune": {"action": "PF-MP (poly, corr, ratio) + gauge, S_det on the gauge scale",
                               "rows": ["gauge", "poly", "corr", "ratio"],
                               "max_force": [round(f, 5) for f in fmax], "mean_force": [round(f, 5) for f in F[:4, 1]],
                               "det_max_force": round(float(F[4, 0]), 5),
                               "rounds": [{"c": round(cc, 6), "steps": st,
                                           "dH2_over_2": round(tuner.mean_dH_estimate([t[0] for t in tr]), 4)}
                                          for cc, st, tr in hist],
                               "tuned_round": best, "steps": steps, "chain": {"n": len(chain), "mean_dH": round(float(np.mean(dH)), 4),
                                                         "acc": float(np.mean(acc)),
                                                         "acc_from_dH2": round(tuner.acceptance_from_dH(tuner.mean_dH_estimate(dH)), 3),
                                                         "nmat": float(np.mean(nmat)),
                                                         "exp_minus_dH": round(float(np.mean(np.exp(-np.array(dH)))), 3)},
                               "cost": round(C, 1), "cost_err": round(dC, 1), "tau_int": tuner.TAU_INT,
                               "seconds": round(time.perf_counter() - t0, 1)}}), flush=True)


def integrator_bench(args):
    """Integrator error against step size for a non-nested and a nested schedule (App. B:
    arbitrary step sizes per term): the PF-MP action in the chosen mixed precision with
    S_det on the gauge scale, step counts (gauge, filter, correction, ratio) scaled by s,
    <dH^2> / 2 over the same 6 inputs at every s, and its exponent in h = 1 / s (4 for a
    second-order integrator, <dH> ~ h^4).  The non-nested base is the tuned schedule of
    --tune; the nested one has step counts dividing each other at similar cost."""
    from paper_1609_02652_amd import synth, tuner
    from paper_1609_02652_amd.pfmp import F16, Lattice
    lat = Lattice(DIMS)
    lat.set_gauge(synth.random_gauge(DIMS, seed=0))
    thermalise(lat, args.therm)
    lat.set_operator(0, KAPPA, CSW)
    lat.set_operator(1, KAPPA_H, CSW)
    log("autotune: %s" % lat.autotune(0))
    bases = {"non_nested": (26, 14, 8, 11), "nested": (28, 14, 7, 14)}
    scales = (1.0, 1.5, 2.0, 3.0)
    out = {}
    for name, base in bases.items():
        rows = []
        for sc in scales:
            n_g, n_p, n_c, n_r = [int(round(b * sc)) for b in base]
            sp = pfmp_spec(lat, steps=dict(poly=n_p, corr=n_c, ratio=n_r, gauge=n_g, det=0), solver_prec=F16)
            U0 = lat.get_gauge().clone()
            dH = []
            for k in range(6):
                P = lat.pack_momenta(synth.gaussian_momenta(lat.V, 9000 + k))
                etas = [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 9100 + 3 * k + j)) for j in range(3)]
                dH.append(lat.trajectory(sp, P, etas, 0.0)["dH"])
                lat.set_gauge(U0)
            m = tuner.mean_dH_estimate(dH)
            rows.append({"scale": sc, "steps": [n_g, n_p, n_c, n_r], "dH2_over_2": round(m, 6),
                         "acc_from_dH2": round(tuner.acceptance_from_dH(m), 3)})
            log("integrator %s %s" % (name, rows[-1]))
        x = np.log([1.0 / r["scale"] for r in rows])
        y = np.log([max(r["dH2_over_2"], 1e-300) for r in rows])
        out[name] = {"rows": rows, "exponent": round(float(np.polyfit(x, y, 1)[0]), 2)}
    lat.close()
    print(json.dumps({"integrator": out, "rows": ["gauge", "poly", "corr", "ratio"]}), flush=True)


def ratio_sweep_bench(args):
    """Integrator error against the ratio of step sizes (App. B: each term on its own,
    arbitrary step size): the PF-MP action in the chosen mixed precision on the dynamically
    thermalised field of --chain's start, the ratio term fixed at n_r steps and the filter
    term at n_r x rho steps for rho from 1 to 6 in steps of 1/2 (integer rho: nested
    schedules; the others interleave), correction and gauge scales fixed; <dH^2>/2 over the
    same 8 inputs at every rho.  An integrator whose error grew with the cross terms of
    non-nested schedules would show jumps at the non-integer rho."""
    from paper_1609_02652_amd import synth, tuner
    from paper_1609_02652_amd.pfmp import F16, Lattice
    lat = Lattice(DIMS)
    lat.set_gauge(synth.random_gauge(DIMS, seed=0))
    thermalise(lat, args.therm)
    lat.set_operator(0, KAPPA, CSW)
    lat.set_operator(1, KAPPA_H, CSW)
    log("autotune: %s" % lat.autotune(0))
    n_g, n_c, n_r = 26, 8, 6
    U0 = lat.get_gauge().clone()
    rows = []
    for twice in range(2, 13):
        rho = twice / 2.0
        n_p = int(round(n_r * rho))
        sp = pfmp_spec(lat, steps=dict(poly=n_p, corr=n_c, ratio=n_r, gauge=n_g, det=0), solver_prec=F16)
        dH, km = [], []
        for k in range(8):
            P = lat.pack_momenta(synth.gaussian_momenta(lat.V, 9300 + k))
            etas = [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 9400 + 3 * k + j)) for j in range(3)]
            st = lat.trajectory(sp, P, etas, 0.0)
            dH.append(st["dH"])
            km.append(st["kmults"])
            lat.set_gauge(U0)
        m = tuner.mean_dH_estimate(dH)
        rows.append({"rho": rho, "steps_gauge_poly_corr_ratio": [n_g, n_p, n_c, n_r], "nested": n_p % n_r == 0,
                     "dH2_over_2": round(m, 6), "acc_from_dH2": round(tuner.acceptance_from_dH(m), 3),
                     "kmults": int(np.mean(km))})
        log("ratio sweep %s" % rows[-1])
    lat.close()
    print(json.dumps({"ratio_sweep": rows}), flush=True)


def chain_bench(args):
    """A Markov chain of PF-MP trajectories in the chosen mixed precision with the tuned step
    counts (gauge, filter, correction, ratio) = (26, 14, 8, 11): after the quenched
    thermalisation, args.chain_therm trajectories with the Metropolis step to bring the field
    into equilibrium with the fermion action, then args.chain trajectories measured: P_acc,
    <exp(-dH)> (1 in equilibrium), N_mat, and the cost C = N_mat / P_acc (eq. cost_func) with
    the error of eq. error_corrected, tau_int measured on the chain (plaquette and accepts)."""
    from paper_1609_02652_amd import synth, tuner
    from paper_1609_02652_amd.pfmp import F16, Lattice
    lat = Lattice(DIMS)
    lat.set_gauge(synth.random_gauge(DIMS, seed=0))
    thermalise(lat, args.therm)
    lat.set_operator(0, KAPPA, CSW)
    lat.set_operator(1, KAPPA_H, CSW)
    log("autotune: %s" % lat.autotune(0))
    steps = tuple(int(v) for v in args.chain_steps.split(","))
    sp = pfmp_spec(lat, steps=dict(gauge=steps[0], poly=steps[1], corr=steps[2], ratio=steps[3], det=0),
                   solver_prec=F16)
    rows = []
    t0 = time.perf_counter()
    for k in range(args.chain_therm + args.chain):
        P = lat.pack_momenta(synth.gaussian_momenta(lat.V, 20000 + k))
        etas = [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 30000 + 3 * k + j)) for j in range(3)]
        st = lat.trajectory(sp, P, etas, float(synth.uniform(40000 + k)[0]))
        plaq = 1.0 - lat.gauge_action(BETA) / (BETA * 6 * lat.V)
        rows.append((st["dH"], int(st["accept"]), st["kmults"], plaq))
        if k % 10 == 0 or k == args.chain_therm + args.chain - 1:
            log("chain %d: dH %.4f accept %d plaquette %.5f (%.0f s)" % (k, st["dH"], st["accept"], plaq,
                                                                         time.perf_counter() - t0))
    lat.close()
    meas = rows[args.chain_therm:]
    dH = np.array([r[0] for r in meas])
    acc = [r[1] for r in meas]
    nmat = [r[2] for r in meas]
    plaq = [r[3] for r in meas]
    tau = max(tuner.tau_int(plaq), tuner.tau_int(acc), 0.5)
    ex = np.exp(-dH)
    C, dC = tuner.cost(nmat, acc, tau)
    out = {"action": "PF-MP (filter p = 4, correction, ratio 0.1300/0.1340) + gauge, S_det on the gauge scale",
           "steps_gauge_poly_corr_ratio": steps, "thermalisation_trajectories": args.chain_therm,
           "measured_trajectories": len(meas), "accept_rate": round(float(np.mean(acc)), 4),
           "exp_minus_dH": round(float(np.mean(ex)), 4),
           "exp_minus_dH_err": round(tuner.corrected_error(ex, tau), 4),
           "mean_dH": round(float(np.mean(dH)), 4), "nmat": round(float(np.mean(nmat)), 1),
           "tau_int_plaquette": round(tuner.tau_int(plaq), 2), "tau_int_accept": round(tuner.tau_int(acc), 2),
           "tau_int_used": round(tau, 2), "cost_C": round(C, 1), "cost_C_err": round(dC, 1),
           "cost_C_rel_err": round(dC / C, 3), "plaquette": round(float(np.mean(plaq)), 6),
           "seconds": round(time.perf_counter() - t0, 1)}
    print(json.dumps({"chain": out}), flush=True)


def config3_bench(args):
    """The batched force-evaluation workload: 24^3 x 48, links relaxed from the seeded start by
    quenched molecular dynamics at beta 5.8, kappa 0.1360, c_sw 1.6, Hasenbusch chain J(0.120)
    K(0.130)^-1 and J(0.130) K(0.136)^-1 with the filter nest (10, 32) on J(0.120) (the nearest
    nested degrees to the workload's 16 / 32: (10 + 1) | (32 + 1)).  One 2MN step of every term at
    tau = 0.02 (three force evaluations of each term at the same links per scale), in four
    forms: FP64 one solve at a time; FP64 with the CG solves due at one merged step batched;
    the chosen mixed precision one at a time (FP16-storage CG with FP64 reliable updates); and
    mixed batched (FP32 batched CG inside FP64 defect correction, multi-RHS stencils sharing
    each link load).  The correction term's z = 0 pole joins the batch in the mixed modes."""
    import torch
    from paper_1609_02652_amd import synth
    from paper_1609_02652_amd.pfmp import Lattice, F64, F16
    dims = (24, 24, 24, 48)
    lat = Lattice(dims)
    out = {"lattice": "x".join(map(str, dims))}
    try:
        lat.set_gauge(synth.random_gauge(dims, seed=0))
        spq = lat.spec(5.8, [], 32, det_op=-1)
        for k in range(args.c3_therm):
            lat.trajectory(spq, lat.pack_momenta(synth.gaussian_momenta(lat.V, 9800 + k)), [], 0.0)
        plaq = 1.0 - lat.gauge_action(5.8) / (5.8 * 6 * lat.V)
        out["thermalisation"] = {"trajectories": args.c3_therm, "gauge_steps": 32, "plaquette": round(plaq, 6)}
        for k, kap in enumerate((0.1360, 0.1200, 0.1300)):
            lat.set_operator(k, kap, CSW)
        out["tuning"] = lat.autotune(0)
        f = lambda kind, n, n1=0: dict(kind=kind, op=1, n=n, n1=n1, mu=1.2, nu=0.9, steps=1)
        terms = [f("poly", 10), f("polyq", 32, 10), f("polycorr", 32),
                 dict(kind="ratio", op=1, op2=2, steps=1), dict(kind="ratio", op=2, op2=0, steps=1)]
        U0 = lat.get_gauge().clone()
        etas = [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 9900 + j)) for j in range(len(terms))]
        phis = lat.heatbath(lat.spec(5.8, terms, 1, det_op=0, solver_prec=F16), etas)
        modes = {"f64_one_by_one": (F64, False), "f64_batched": (F64, True),
                 "mixed_one_by_one": (F16, False), "mixed_batched": (F16, True)}
        for name, (prec, batch) in list(modes.items()) * 2:   # the second pass of each is kept
            sp = lat.spec(5.8, terms, 1, det_op=0, tau=0.02, batch=batch, solver_prec=prec)
            P = lat.pack_momenta(synth.gaussian_momenta(lat.V, 9990))
            lat.set_gauge(U0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = lat.md_evolve(sp, P, phis)
            torch.cuda.synchronize()
            out[name] = {"s": round(time.perf_counter() - t0, 4), "solver_iters": st["solver_iters"],
                         "kmults": st["kmults"]}
            log("config3 %s: %s" % (name, out[name]))
        out["batched_speedup_f64"] = round(out["f64_one_by_one"]["s"] / out["f64_batched"]["s"], 3)
        out["batched_speedup_mixed"] = round(out["mixed_one_by_one"]["s"] / out["mixed_batched"]["s"], 3)
        out["chosen_vs_plain_f64"] = round(out["f64_one_by_one"]["s"] /
                                           min(out["mixed_one_by_one"]["s"], out["mixed_batched"]["s"]), 3)
    finally:
        lat.close()
    print(json.dumps({"config3": out}), flush=True)


# ---- the light-quark trajectory workload: 48^3 x 96, beta 5.9, kappa 0.1370, c_sw 1.6,
# Hasenbusch masses 0.120 / 0.130 / 0.135, filter nest (6, 20, 62) on J(0.120) (the nearest
# degrees with the nested factorisation (p1 + 1) | (p2 + 1) that the workload's 16/32/64 lack),
# four integrator scales, tau = 1, every solve to 1e-10.
C5_DIMS = (48, 48, 48, 96)
C5_BETA, C5_KAPPA, C5_CSW = 5.9, 0.1370, 1.6
C5_HASEN = (0.120, 0.130, 0.135)
C5_NEST = (6, 20, 62)


def config5_spec(lat, steps, tol=TOL, **kw):
    """Slots 0 = K (0.1370), 1 = J (0.120, the filter nest), 2 = 0.130, 3 = 0.135.  Scales
    (steps = gauge, filter, correction, ratios): {gauge + S_det}, {P_6, Q(20/6), Q(62/20)},
    {correction [J P_62(J)]^-1, ratio J(0.120)/K(0.130)}, {ratios 0.130/0.135 and 0.135/0.1370}."""
    n_g, n_p, n_c, n_r = steps[:4]
    n_l = steps[4] if len(steps) > 4 else n_r   # optional: the lightest ratio on a scale of its own
    p1, p2, p3 = C5_NEST
    f = lambda kind, n, st, n1=0: dict(kind=kind, op=1, n=n, n1=n1, mu=1.2, nu=0.9, steps=st)
    terms = [f("poly", p1, n_p), f("polyq", p2, n_p, p1), f("polyq", p3, n_p, p2), f("polycorr", p3, n_c),
             dict(kind="ratio", op=1, op2=2, steps=n_c), dict(kind="ratio", op=2, op2=3, steps=n_r),
             dict(kind="ratio", op=3, op2=0, steps=n_l)]
    return lat.spec(C5_BETA, terms, n_g, det_op=0, tol=tol, **kw)


def config5_action_check(lat, steps, P, ed):
    """Accuracy of the action evaluation at this volume: the heatbath (chosen solver, the
    trajectories' tolerance) makes S_j(phi_j) = eta_j^dag eta_j; each S_j is then evaluated
    with plain FP64 solves to 1e-10 and 1e-13 and with the chosen solver to 1e-10."""
    from paper_1609_02652_amd.pfmp import F64, F16
    eta2 = [lat.dot(e, e).real for e in ed]
    phis = lat.heatbath(config5_spec(lat, steps, solver_prec=F16), ed)
    out = {"eta_dag_eta": eta2}
    for name, tol, prec in (("plain_f64_1e-10", 1e-10, F64), ("chosen_1e-10", 1e-10, F16),
                            ("plain_f64_1e-13", 1e-13, F64)):
        _, parts = lat.hamiltonian(config5_spec(lat, steps, tol=tol, solver_prec=prec), P, phis)
        d = [a - b for a, b in zip(parts[3:], eta2)]
        out[name] = {"S_minus_eta_dag_eta": d, "max_abs": max(abs(v) for v in d)}
        log("config5 actions, %s: max |S_j - eta_j^dag eta_j| = %.3g" % (name, out[name]["max_abs"]))
    return out


def config5_bench(args):
    """One timed trajectory per mode (plain FP64 CG form; the chosen mixed-precision form) of
    the light-quark workload from the same thermalised field and the same momenta, noise and
    Metropolis uniform."""
    import torch
    from paper_1609_02652_amd import synth
    from paper_1609_02652_amd.pfmp import Lattice, F64, F16
    steps = tuple(int(v) for v in args.c5_steps.split(","))
    dims = tuple(int(v) for v in args.c5_dims.split(","))
    out = {"lattice": "x".join(map(str, dims)), "steps_gauge_filter_corr_ratio": steps, "tau": args.c5_tau,
           "tol": args.c5_tol}
    t0 = time.perf_counter()
    U = synth.random_gauge(dims, seed=0)
    log("config5: seeded start field %.1f s" % (time.perf_counter() - t0))
    lat = Lattice(dims)
    lat.verbose(1)
    lat.set_gauge(U)
    lat.set_operator(0, C5_KAPPA, C5_CSW)
    # (parity of this lattice against the oracle on sampled sites is a GPU test:
    # tests/test_gpu_bench_shapes.py, test_operator_sampled_at_light_quark_shape)
    del U
    # quenched thermalisation at beta 5.9: molecular dynamics trajectories, every one kept
    sp_q = lat.spec(C5_BETA, [], args.c5_therm_steps, det_op=-1)
    t0 = time.perf_counter()
    for k in range(args.c5_therm):
        st = lat.trajectory(sp_q, lat.pack_momenta(synth.gaussian_momenta(lat.V, 9000 + k)), [], 0.0)
        plaq = 1.0 - lat.gauge_action(C5_BETA) / (C5_BETA * 6 * lat.V)
        log("config5 thermalisation %d: dH %.2f plaquette %.5f" % (k, st["dH"], plaq))
    out["thermalisation"] = {"trajectories": args.c5_therm, "gauge_steps": args.c5_therm_steps,
                             "accept": "all (molecular-dynamics relaxation)", "plaquette": round(plaq, 6),
                             "seconds": round(time.perf_counter() - t0, 1)}
    for k, kap in enumerate(C5_HASEN):
        lat.set_operator(1 + k, kap, C5_CSW)
    out["autotune"] = lat.autotune(0)
    log("config5 autotune %s" % out["autotune"])
    # FP16-storage solver with FP16 or FP32 copies of links and clover: the faster on one solve at 0.1370
    b = lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 2))
    hl = {}
    for on in (1, 0):
        lat.half_links(on)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = lat.cg_solve(0, b, tol=TOL, prec=F16, maxiter=100000)
        torch.cuda.synchronize()
        hl[on] = (time.perf_counter() - t0, st["iters"])
        log("config5 fp16-storage CG at kappa 0.1370, half links %d: %.2f s, %d iterations" % (on, *hl[on]))
    half = 1 if hl[1][0] <= hl[0][0] else 0
    lat.half_links(half)
    out["cg_f16_kappa_0.1370"] = {"half_links_1": {"s": round(hl[1][0], 3), "iters": hl[1][1]},
                                  "half_links_0": {"s": round(hl[0][0], 3), "iters": hl[0][1]}, "chosen": half}
    # optional relaxation with the fermions: molecular-dynamics trajectories of the full action
    # (chosen mode, the timed trajectories' steps and length, every one kept), so that the timed
    # ones start nearer the equilibrium of the dynamical action than the quenched field does
    if args.c5_dyn_therm:
        sp_d = config5_spec(lat, steps, tol=args.c5_tol, tau=args.c5_tau, solver_prec=F16)
        t0 = time.perf_counter()
        for k in range(args.c5_dyn_therm):
            # heatbath, then the molecular dynamics alone: the evolved field is kept whatever dH
            phis_k = lat.heatbath(sp_d, [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 9200 + 7 * k + j))
                                         for j in range(7)])
            st = lat.md_evolve(sp_d, lat.pack_momenta(synth.gaussian_momenta(lat.V, 9100 + k)), phis_k)
            del phis_k
            plaq = 1.0 - lat.gauge_action(C5_BETA) / (C5_BETA * 6 * lat.V)
            log("config5 relaxation with the fermions %d: %d solver iterations, plaquette %.5f"
                % (k, st["solver_iters"], plaq))
        out["dynamical_relaxation"] = {"trajectories": args.c5_dyn_therm, "plaquette": round(plaq, 6),
                                       "seconds": round(time.perf_counter() - t0, 1)}
    U0 = lat.get_gauge().clone()
    P = synth.gaussian_momenta(lat.V, 9500)
    etas = [synth.gaussian_spinor(lat.Vh, 9600 + j) for j in range(7)]
    u = float(synth.uniform(9700)[0])
    # plain FP64 against the chosen form at this size without a whole trajectory: one CG solve
    # on K(0.1370), and one force evaluation of every row of the action (all its solves) at
    # the thermalised field with the heatbath's pseudofermions
    cmp = {}
    for name, prec in (() if args.c5_no_compare else (("plain_f64", F64), ("chosen", F16))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = lat.cg_solve(0, b, tol=TOL, prec=prec, maxiter=100000)
        torch.cuda.synchronize()
        cmp["cg_kappa_0.1370_" + name] = {"s": round(time.perf_counter() - t0, 3), "iters": st["iters"],
                                          "true_res": st["true_res"]}
        log("config5 CG %s: %s" % (name, cmp["cg_kappa_0.1370_" + name]))
    ed = [lat.pack_spinor(e) for e in etas]
    phis = lat.heatbath(config5_spec(lat, steps, solver_prec=F16), ed) if not args.c5_no_compare else None
    for name, kw in (() if args.c5_no_compare else (("plain_f64", {}), ("chosen", dict(solver_prec=F16)))):
        sp = config5_spec(lat, steps, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn = lat.force_norms(sp, phis)
        torch.cuda.synchronize()
        cmp["force_evaluation_" + name] = {"s": round(time.perf_counter() - t0, 3),
                                           "max_force_rows": [round(float(v), 4) for v in fn[:, 0]]}
        log("config5 force evaluation %s: %s" % (name, cmp["force_evaluation_" + name]))
    if cmp:
        cmp["cg_speedup"] = round(cmp["cg_kappa_0.1370_plain_f64"]["s"] / cmp["cg_kappa_0.1370_chosen"]["s"], 3)
        cmp["force_evaluation_speedup"] = round(cmp["force_evaluation_plain_f64"]["s"] /
                                                cmp["force_evaluation_chosen"]["s"], 3)
        out["fp64_vs_chosen"] = cmp
    del ed, phis
    if args.c5_action_check:
        out["action_check"] = config5_action_check(lat, steps, lat.pack_momenta(P),
                                                   [lat.pack_spinor(e) for e in etas])
    torch.cuda.empty_cache()
    modes = [("chosen", dict(solver_prec=F16)), ("plain_f64", {})]
    if args.c5_modes != "both":
        modes = [m for m in modes if m[0] == args.c5_modes]
    out["trajectory"] = {}
    for name, kw in modes:
        lat.set_gauge(U0)
        sp = config5_spec(lat, steps, tol=args.c5_tol, tau=args.c5_tau, **kw)
        Pd = lat.pack_momenta(P)
        ed = [lat.pack_spinor(e) for e in etas]
        torch.cuda.empty_cache()   # the library allocates outside torch's cache
        log("config5 trajectory, %s" % name)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = lat.trajectory(sp, Pd, ed, u)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["trajectory"][name] = {"s": round(dt, 2), "dH": st["dH"], "accept": st["accept"],
                                   "kmults": st["kmults"], "solver_iters": st["solver_iters"],
                                   "nforce": list(st["nforce"][:8]), "H0": st["H0"],
                                   # change of each part of H (kinetic, S_G, S_det, the terms)
                                   "dparts": [b - a for a, b in zip(st["parts0"], st["parts1"])]}
        log("config5 %s: %.1f s, dH %.4f, accept %d, %d Khat multiplications" % (name, dt, st["dH"], st["accept"],
                                                                                st["kmults"]))
    if "chosen" in out["trajectory"] and "plain_f64" in out["trajectory"]:
        c, f = out["trajectory"]["chosen"], out["trajectory"]["plain_f64"]
        out["speedup_chosen_vs_f64"] = round(f["s"] / c["s"], 3)
        out["dH_difference"] = c["dH"] - f["dH"]
    lat.close()
    print(json.dumps({"config5": out}), flush=True)


def run_trajectories(lat, sp, steps, warmup, seed):
    """warmup untimed, then exactly `steps` timed trajectories on fresh momenta and
    pseudofermion sources; the links are restored after each so every mode sees
    the same starting configuration."""
    import torch
    from paper_1609_02652_amd import synth
    V, Vh = lat.V, lat.Vh
    U0 = lat.get_gauge().clone()

    def inputs(k):
        P = lat.pack_momenta(synth.gaussian_momenta(V, seed + k))
        etas = [lat.pack_spinor(synth.gaussian_spinor(Vh, seed + 10000 + 3 * k + j)) for j in range(sp.nterms)]
        return P, etas

    for k in range(warmup):
        P, etas = inputs(k)
        st = lat.trajectory(sp, P, etas, synth.uniform(seed + k)[0])
        log("warmup traj %d: dH %.4f %.3f s" % (k, st["dH"], st["seconds"]))
        lat.set_gauge(U0)
    batch = [inputs(1000 + k) for k in range(steps)]
    us = [synth.uniform(seed + 500 + k)[0] for k in range(steps)]
    stats, elapsed = [], 0.0
    for k in range(steps):
        P, etas = batch[k]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats.append(lat.trajectory(sp, P, etas, us[k]))
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        lat.set_gauge(U0)
    for st in stats:
        log("traj: dH %.5f accept %d %.3f s kmults %d iters %d nforce %s"
            % (st["dH"], st["accept"], st["seconds"], st["kmults"], st["solver_iters"], st["nforce"]))
    return elapsed / steps, stats


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32, help="timed solves (sources) per precision")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--therm", type=int, default=20, help="quenched thermalisation trajectories")
    ap.add_argument("--roofline-only", action="store_true",
                    help="time only the hopping kernels and a plain copy (for counter runs)")
    ap.add_argument("--batch-only", action="store_true",
                    help="time only the multi-RHS Khat comparison at 32^3 x 64 and a plain copy (for counter runs)")
    ap.add_argument("--batch-zt", help="with --batch-only: repeat the comparison under these site visit orders, "
                                       "e.g. 0,1,2,4,8,16")
    ap.add_argument("--tune", action="store_true",
                    help="the paper's step-size tuning (F_i h_i = const, P_acc in [0.65, 0.75]) and cost "
                         "C = N_mat / P_acc for the PF-MP action")
    ap.add_argument("--learned32", action="store_true",
                    help="the learned preconditioner trained and used at 32^3 x 64 against plain and mixed CG")
    ap.add_argument("--integrator", action="store_true",
                    help="<dH^2>/2 against the step scale for a non-nested and a nested PF-MP schedule")
    ap.add_argument("--zoo", action="store_true",
                    help="one trajectory of each of the paper's actions (PF-MP, 1MP, 2MP, 1PF, 2PF, 2PF-1MP, "
                         "1PF-2MP) in FP64 and in the chosen mixed precision")
    ap.add_argument("--cg-lattice", help="only the CG iteration roofline (FP64, FP32, FP16 storage) on this "
                                          "lattice, e.g. 32,32,32,64 (seeded start field; for kernel profiles)")
    ap.add_argument("--config3", action="store_true",
                    help="the batched force-evaluation workload at 24^3 x 48 (one 2MN step, four forms)")
    ap.add_argument("--c3-therm", type=int, default=20, help="quenched relaxation trajectories at beta 5.8")
    ap.add_argument("--ratio-sweep", action="store_true",
                    help="<dH^2>/2 against the filter / ratio step-size ratio (nested and interleaved schedules)")
    ap.add_argument("--chain", type=int, default=0,
                    help="a Markov chain of this many measured PF-MP trajectories (P_acc, <exp(-dH)>, cost C)")
    ap.add_argument("--chain-therm", type=int, default=20, help="Metropolis trajectories before measuring")
    ap.add_argument("--chain-steps", default="26,14,8,11", help="2MN steps: gauge, filter, correction, ratio")
    ap.add_argument("--config5", action="store_true",
                    help="the light-quark trajectory workload at 48^3 x 96: one trajectory per mode")
    ap.add_argument("--c5-steps", default="24,8,4,3", help="2MN steps: gauge, filter, correction, ratios")
    ap.add_argument("--c5-dims", default=",".join(map(str, C5_DIMS)), help="lattice (a smaller one for a dry run)")
    ap.add_argument("--c5-therm", type=int, default=20, help="quenched thermalisation trajectories")
    ap.add_argument("--c5-therm-steps", type=int, default=64, help="2MN steps of a thermalisation trajectory")
    ap.add_argument("--c5-modes", default="both", choices=["both", "chosen", "plain_f64", "none"])
    ap.add_argument("--c5-tau", type=float, default=1.0, help="trajectory length of the timed trajectories")
    ap.add_argument("--c5-tol", type=float, default=TOL, help="relative residual of every solve of the timed "
                                                              "trajectories")
    ap.add_argument("--c5-dyn-therm", type=int, default=0,
                    help="molecular-dynamics trajectories of the full action (chosen mode, every one kept) "
                         "before the timed ones")
    ap.add_argument("--c5-action-check", action="store_true",
                    help="after the set-up: each action term at the heatbath field solved to 1e-10 and 1e-13 "
                         "against eta^dag eta")
    ap.add_argument("--c5-no-compare", action="store_true",
                    help="skip the FP64-against-chosen CG and force-evaluation comparison")
    ap.add_argument("--cpu-full", action="store_true",
                    help="the oracle on the host: a full solve and the 4^4 trajectory, 1 thread and all threads")
    ap.add_argument("--cpu-child", choices=["cg", "traj"], help=argparse.SUPPRESS)
    ap.add_argument("--trajectory-only", choices=["f64", "f32", "f16"],
                    help="thermalise, then run --warmup and --steps trajectories in one solver precision and "
                         "print their times (for kernel profiles of one trajectory)")
    args = ap.parse_args()
    if args.cpu_child:
        r = oracle_cg_solve() if args.cpu_child == "cg" else oracle_config1_trajectory()
        print(json.dumps(dict(r, threads=int(os.environ.get("OMP_NUM_THREADS", "0")))), flush=True)
        return
    if args.cpu_full:
        cpu_full(args)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.roofline_only:
        roofline_only(max(args.steps, 10))
        return
    if args.batch_only:
        batch_only(max(args.steps, 10), [int(v) for v in args.batch_zt.split(",")] if args.batch_zt else None)
        return
    if args.zoo:
        zoo_bench(args)
        return
    if args.tune:
        tune_bench(args)
        return
    if args.integrator:
        integrator_bench(args)
        return
    if args.learned32:
        learned32_bench(args)
        return
    if args.config5:
        config5_bench(args)
        return
    if args.cg_lattice:
        dims = tuple(int(v) for v in args.cg_lattice.split(","))
        from paper_1609_02652_amd import synth
        lt = make_lattice(dims, synth.random_gauge(dims, seed=5))
        tune = lt.autotune(0)
        r = cg_iteration_roofline(lt, lt.Vh)
        lt.close()
        # a 256 MiB copy of known size in the same run calibrates FETCH_SIZE / WRITE_SIZE
        print(json.dumps({"cg_iteration_roofline": r, "lattice": args.cg_lattice, "tuning": tune,
                          "copy_256MiB": copy_bandwidth()}), flush=True)
        return
    if args.config3:
        config3_bench(args)
        return
    if args.ratio_sweep:
        ratio_sweep_bench(args)
        return
    if args.chain > 0:
        chain_bench(args)
        return
    from paper_1609_02652_amd import synth
    from paper_1609_02652_amd.pfmp import F64, F32, F16, Lattice
    if args.trajectory_only:
        lat = Lattice(DIMS)
        lat.set_gauge(synth.random_gauge(DIMS, seed=0))
        thermalise(lat, args.therm)
        lat.set_operator(0, KAPPA, CSW)
        lat.set_operator(1, KAPPA_H, CSW)
        log("autotune: %s" % lat.autotune(0))
        prec = {"f64": F64, "f32": F32, "f16": F16}[args.trajectory_only]
        sp = pfmp_spec(lat, solver_prec=prec)
        t, sts = run_trajectories(lat, sp, args.steps, args.warmup, 100)
        lat.close()
        print(json.dumps({"trajectory_only": args.trajectory_only, "s_per_traj": round(t, 4),
                          "kmults": [s["kmults"] for s in sts], "dH": [round(s["dH"], 5) for s in sts]}), flush=True)
        return
    log("bench: building inputs", DIMS)
    lat = Lattice(DIMS)
    lat.set_gauge(synth.random_gauge(DIMS, seed=0))
    therm = thermalise(lat, args.therm)
    lat.set_operator(0, KAPPA, CSW)
    lat.set_operator(1, KAPPA_H, CSW)
    tune = lat.autotune(0)
    log("autotune: %s" % tune)

    # ---- the headline: CG solves of the solve workload at 1e-10, warmup then exactly `steps`
    # sources timed in each precision; the chosen form is the faster mixed-precision one
    cg = cg_bench(lat, args.steps, args.warmup)
    cg["roofline_16x16x16x32"] = cg_roofline(cg, lat.Vh)
    chosen = min(("f32", "f16"), key=lambda k: cg[k]["mean_s"])
    t_chosen = cg[chosen]["mean_s"]

    # ---- context on the same field: the batched Hasenbusch-chain solve, the learned
    # preconditioner, and the 16^3 x 32 PF-MP trajectory of the previous headline
    lat.set_operator(2, 0.1250, CSW)
    batched = batch_bench(lat)
    learned, _ = learned_bench(lat, 8)
    learned["speedup_vs_f64_cg"] = round(cg["f64"]["median_s"] / learned["fcg_median_s"], 3)
    learned["iters_saved_vs_f64_cg"] = round(1 - learned["fcg_iters"] / cg["f64"]["iters"], 3)
    traj16 = {}
    for name, kw in (("plain_f64", {}), ("chosen", {"solver_prec": F16 if chosen == "f16" else F32})):
        t, sts = run_trajectories(lat, pfmp_spec(lat, **kw), 1, 1 if name == "chosen" else 0, 100)
        traj16[name] = {"s_per_traj": round(t, 3), "dH": round(sts[0]["dH"], 5), "accept": sts[0]["accept"],
                        "kmults": sts[0]["kmults"]}
    traj16["speedup"] = round(traj16["plain_f64"]["s_per_traj"] / traj16["chosen"]["s_per_traj"], 3)
    lat.close()

    # ---- the correctness-workload trajectory (4^4, kappa 0.120 / 0.110, degree-4 filter)
    # in the plain FP64 form and the chosen form, on the same inputs
    traj1 = config1_trajectories(F16 if chosen == "f16" else F32, args.warmup)

    # ---- dominant-kernel roofline (HIP events on the library stream).  The hop is
    # priced at the algorithmic bytes of one hop per output site, links as 8 x 18 reals
    # plus the input and output spinors (1,536 B in FP64); the kernel itself reads SU(3)
    # links as 2 rows (12 reals), so the bytes it must move are 1,152 B per site, also
    # reported.  The HBM figure is taken at 32^3 x 64, whose working set is far larger
    # than the 256 MB Infinity Cache; the same lattice gives the CG iteration's roofline
    # in each precision and the multi-RHS Khat.
    def roof_entry(dims, r):
        key = "x".join(map(str, dims))
        algo = r["Vh"] * (8 * 18 + 24 + 24) * 8
        moved = r["bytes_hop"]
        return {"lattice": key, "avg_launch_us": round(r["t_hop"] * 1e6, 2), "bytes_per_launch": algo,
                "achieved": round(algo / r["t_hop"] / 1e9, 1), "frac": round(algo / r["t_hop"] / 1e9 / HBM_PEAK_GBS, 4),
                "moved_bytes_per_launch": moved, "achieved_moved": round(moved / r["t_hop"] / 1e9, 1),
                "frac_moved": round(moved / r["t_hop"] / 1e9 / HBM_PEAK_GBS, 4),
                "Mhat_us": round(r["t_M"] * 1e6, 2), "Mhat_GBps": round(r["bytes_M"] / r["t_M"] / 1e9, 1),
                "tuning": r["tune"], "traffic": pmc_traffic(key)}

    big = (32, 32, 32, 64)
    extra32 = {}

    def big_extra(lt):
        extra32["cg_iteration_roofline"] = cg_iteration_roofline(lt, lt.Vh)
        extra32["multi_rhs_Khat"] = batch_apply(lt)
        return None

    rb = hop_roofline(big, synth.random_gauge(big, seed=5), reps=50, extra=big_extra)
    main_e = roof_entry(big, rb)
    roof = {"kernel": "hop D_oe, FP64 (k_hop_clovinv, plain), %s" % main_e["lattice"], "bound": "hbm",
            "achieved": main_e["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": main_e["frac"],
            "traffic": main_e["traffic"]}
    roof.update({k: v for k, v in main_e.items() if k not in roof})
    roof["bytes_basis"] = ("algorithmic: links 8 x 18 + spinor in 24 + out 24 reals per output site (FP64); "
                           "moved: links read as 12 reals")
    roof["copy"] = copy_bandwidth()
    roof["cg_iteration_32x32x32x64"] = extra32.get("cg_iteration_roofline")

    out = {
        "metric": "PF-MP trajectory s & CG solve s at 1e-10 resid, plain FP64 vs chosen; Dslash GB/s",
        "value": round(t_chosen, 6),
        "unit": "s/solve",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_chosen * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32+f64", "f16": "f16-storage/f32+f64"}[chosen],
        "data": "synthetic",
        "config": {"workload": "mixed-precision solve benchmark: 16^3x32, links from %d quenched HMC "
                               "trajectories at beta=5.7 from the seeded start, even-odd clover kappa=0.1340 "
                               "c_sw=1.6, Gaussian sources one at a time, CG on Mhat^dag Mhat to 1e-10 with "
                               "FP64 reliable updates; one step = one solve" % args.therm,
                   "lattice": "16x16x16x32",
                   "mode": "chosen (the faster measured): %s" % {
                       "f32": "FP32 inner CG with FP64 reliable updates",
                       "f16": "FP32 arithmetic with FP16 spinor storage, FP64 reliable updates"}[chosen]},
        "cg_solve": dict(cg, tol=TOL, sources=args.steps, chosen=chosen,
                         speedup_chosen_vs_f64=round(cg["f64"]["mean_s"] / t_chosen, 3)),
        "trajectory": {
            "light_quark_48x48x48x96": "not in this line (7-14 minutes per trajectory): bench.py --config5, "
                                       "plain FP64 and chosen trajectories with dH and the accept decisions "
                                       "in profiles/config5_trajectory_48x48x48x96.md",
            "markov_chain_16x16x16x32": "not in this line (300 trajectories, 6 minutes): bench.py --chain 300, "
                                        "P_acc, <exp(-dH)> and the cost C in profiles/pfmp_chain_16x16x16x32.md",
            "correctness_workload_4x4x4x4": traj1,
            "pfmp_16x16x16x32_context": traj16},
        "multi_rhs_Khat_32x32x32x64": extra32.get("multi_rhs_Khat"),
        "batched_chain_cg_16x16x16x32": batched,
        "learned_preconditioner_16x16x16x32": learned,
        "paper_context": {
            "note": "the paper publishes work counts only (K multiplications per trajectory over acceptance), on "
                    "its own 16^3x32 Wilson ensemble at kappa 0.15825 with a modified BQCD; hardware, precision "
                    "and times are not stated; context, not a target",
            "cost_C_PF-MP": "29000 +- 1800 (Table 3.6, p = 4, kappa' = 0.155, steps (6, 20, 120, 480))",
            "cost_C_2MP": "31000 +- 2200 (Table 3.5)",
            "kmults_per_filter_force": "2p - 2 (Table 3.2)"},
        "thermalisation": therm,
        "autotune": tune,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def config1_trajectories(prec, warmup, steps=3):
    """The correctness workload's trajectory (4^4, periodic space, antiperiodic time; beta 5.6;
    kappa 0.120, c_sw 1.0; Hasenbusch kappa' 0.110; degree-4 filter; 2MN steps (ratio,
    correction, filter, gauge) = (10, 20, 40, 80); CG 1e-12) in the plain FP64 form and the
    chosen form on the same seeded inputs: seconds per trajectory, dH and accept."""
    import torch
    from paper_1609_02652_amd import synth
    from paper_1609_02652_amd.pfmp import Lattice
    dims = (4, 4, 4, 4)
    out = {}
    for name, kw in (("plain_f64", {}), ("chosen", {"solver_prec": prec})):
        lat = Lattice(dims)
        lat.set_gauge(synth.random_gauge(dims, seed=0))
        lat.set_operator(0, 0.120, 1.0)
        lat.set_operator(1, 0.110, 1.0)
        terms = [dict(kind="poly", op=1, n=4, mu=1.2, nu=0.9, steps=40),
                 dict(kind="polycorr", op=1, n=4, mu=1.2, nu=0.9, steps=20),
                 dict(kind="ratio", op=1, op2=0, steps=10)]
        sp = lat.spec(5.6, terms, 80, det_op=0, tol=1e-12, **kw)
        U0 = lat.get_gauge().clone()
        sts, tot = [], 0.0
        for k in range(warmup + steps):
            P = lat.pack_momenta(synth.gaussian_momenta(lat.V, 100 + k))
            etas = [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 20 + 3 * k + j)) for j in range(3)]
            lat.set_gauge(U0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = lat.trajectory(sp, P, etas, float(synth.uniform(200 + k)[0]))
            torch.cuda.synchronize()
            if k >= warmup:
                tot += time.perf_counter() - t0
                sts.append(st)
        lat.close()
        out[name] = {"s_per_traj": round(tot / steps, 4), "dH": [round(st["dH"], 10) for st in sts],
                     "accept": [int(st["accept"]) for st in sts]}
    out["speedup"] = round(out["plain_f64"]["s_per_traj"] / out["chosen"]["s_per_traj"], 3)
    out["same_accept_decisions"] = out["plain_f64"]["accept"] == out["chosen"]["accept"]
    return out


if __name__ == "__main__":
    main()
