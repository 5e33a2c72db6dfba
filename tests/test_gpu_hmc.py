"""PF-MP HMC on the GPU against the oracle (through the C-ABI): heatbath identity,
one full trajectory of the 4^4 correctness workload (paper eq. pfmp_action with
the App. B integrator), reversibility, dH ~ h^2 and <exp(-dH)> = 1."""
import math

import numpy as np
import pytest

import oracle
from oracle import hmc
from paper_1609_02652_amd import synth

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 4, 4)
KAPPA, KAPPA_H, CSW, BETA = 0.120, 0.110, 1.0, 5.6


def gpu_spec(lat, steps=(10, 20, 40, 80), tol=1e-12, exact_start=True, terms=(0, 1, 2)):
    n_jk, n_corr, n_p, n_g = steps
    allt = [dict(kind="poly", op=1, n=4, mu=1.2, nu=0.9, steps=n_p),
            dict(kind="polycorr", op=1, n=4, mu=1.2, nu=0.9, steps=n_corr),
            dict(kind="ratio", op=1, op2=0, steps=n_jk)]
    return lat.spec(BETA, [allt[i] for i in terms], n_g, det_op=0, tol=tol, exact_start=exact_start)


def oracle_spec(steps=(10, 20, 40, 80), terms=(0, 1, 2)):
    n_jk, n_corr, n_p, n_g = steps
    allt = [dict(kind="poly", kappa=KAPPA_H, n=4, mu=1.2, nu=0.9, steps=n_p),
            dict(kind="polycorr", kappa=KAPPA_H, n=4, mu=1.2, nu=0.9, steps=n_corr),
            dict(kind="ratio", kappa_num=KAPPA_H, kappa_den=KAPPA, steps=n_jk)]
    return dict(dims=DIMS, beta=BETA, csw=CSW, kappa=KAPPA, gauge_steps=n_g, terms=[allt[i] for i in terms])


def make_lattice(U):
    from paper_1609_02652_amd.pfmp import Lattice
    lat = Lattice(DIMS)
    lat.set_gauge(U)
    lat.set_operator(0, KAPPA, CSW)
    lat.set_operator(1, KAPPA_H, CSW)
    return lat


@pytest.fixture(scope="module")
def U0():
    return synth.random_gauge(DIMS, seed=0)


def test_heatbath_matches_oracle(U0):
    lat = make_lattice(U0)
    sp = gpu_spec(lat)
    etas = [synth.gaussian_spinor(lat.Vh, 20 + j) for j in range(3)]
    phis = lat.heatbath(sp, [lat.pack_spinor(e) for e in etas])
    P = lat.pack_momenta(synth.gaussian_momenta(lat.V, 100))
    H, parts = lat.hamiltonian(sp, P, phis)
    ops = hmc.Ops(DIMS, U0, CSW)
    ospec = oracle_spec()
    for j, t in enumerate(ospec["terms"]):
        e2 = np.vdot(etas[j], etas[j]).real
        assert abs(parts[3 + j] - e2) < 1e-9 * e2, (j, parts[3 + j], e2)
        phi_o = hmc.heatbath(ops, t, etas[j])
        assert np.linalg.norm(lat.spinor_numpy(phis[j]) - phi_o) / np.linalg.norm(phi_o) < 1e-9
    lat.close()


def test_force_norms_match_oracle(U0):
    """Force sizes for step tuning (Sec. 2.4): max and mean over links of the coefficient norm
    of the gauge force, each PF-MP term's force and the S_det force, against the oracle's
    forces for the same eta (its own heatbath)."""
    lat = make_lattice(U0)
    sp = gpu_spec(lat)
    etas = [synth.gaussian_spinor(lat.Vh, 20 + j) for j in range(3)]
    phis = lat.heatbath(sp, [lat.pack_spinor(e) for e in etas])
    got = lat.force_norms(sp, phis)
    ops = hmc.Ops(DIMS, U0, CSW)
    Fs = [oracle.force_gauge(DIMS, U0, BETA)]
    for j, t in enumerate(oracle_spec()["terms"]):
        Fs.append(hmc.force(ops, t, hmc.heatbath(ops, t, etas[j]), 1e-13))
    Fd = np.zeros_like(Fs[0])
    ops(KAPPA).force_logdet(Fd)
    Fs.append(Fd)
    assert got.shape == (len(Fs), 2)
    for row, F in enumerate(Fs):
        nrm = np.sqrt((F ** 2).sum(axis=2))
        print("row", row, got[row], nrm.max(), nrm.mean(), flush=True)
        assert abs(got[row, 0] - nrm.max()) < 1e-8 * nrm.max()
        assert abs(got[row, 1] - nrm.mean()) < 1e-8 * nrm.mean()
    lat.close()


def test_trajectory_matches_oracle(U0):
    """4^4, kappa 0.120 / 0.110, c_sw 1.0, degree-4 filter, 2MN steps (10, 20, 40, 80), CG 1e-12."""
    print("trajectory 4^4 config", flush=True)
    P0 = synth.gaussian_momenta(256, 100)
    etas = [synth.gaussian_spinor(128, 20 + j) for j in range(3)]
    u = synth.uniform(200)[0]
    ref = hmc.trajectory(oracle_spec(), U0, P0, etas, u=u, tol=1e-12)
    lat = make_lattice(U0)
    sp = gpu_spec(lat)
    Pend = lat.pack_momenta(np.zeros((256, 4, 8)))
    st = lat.trajectory(sp, lat.pack_momenta(P0), [lat.pack_spinor(e) for e in etas], u, P_end=Pend)
    print("dH gpu %.12f oracle %.12f" % (st["dH"], ref["dH"]), st["nforce"], ref["nforce"], flush=True)
    assert st["nforce"] == ref["nforce"]
    assert abs(st["H0"] - ref["H0"]) < 1e-8 * abs(ref["H0"])
    Ug = lat.get_gauge().cpu().numpy()
    Pg = lat.unpack_momenta(Pend).cpu().numpy()
    print("|dH - dH_oracle| %.2e, max |U - U_oracle| %.2e, max |P - P_oracle| %.2e"
          % (abs(st["dH"] - ref["dH"]), np.max(np.abs(Ug - ref["U"])), np.max(np.abs(Pg - ref["P"]))), flush=True)
    assert abs(st["dH"] - ref["dH"]) < 1e-10
    assert st["accept"] == ref["accept"]
    if st["accept"]:
        assert np.max(np.abs(Ug - ref["U"])) < 1e-10
    else:
        assert np.array_equal(Ug, U0)
    assert np.max(np.abs(lat.unpack_momenta(Pend).cpu().numpy() - ref["P"])) < 1e-8
    lat.close()


def test_reversibility_gpu(U0):
    lat = make_lattice(U0)
    sp = gpu_spec(lat, steps=(3, 5, 7, 11), tol=1e-13)
    etas = [lat.pack_spinor(synth.gaussian_spinor(lat.Vh, 30 + j)) for j in range(3)]
    phis = lat.heatbath(sp, etas)
    P0 = synth.gaussian_momenta(lat.V, 101)
    P = lat.pack_momenta(P0)
    lat.md_evolve(sp, P, phis)
    assert np.max(np.abs(lat.get_gauge().cpu().numpy() - U0)) > 1e-2
    P.neg_()
    lat.md_evolve(sp, P, phis)
    assert np.max(np.abs(lat.get_gauge().cpu().numpy() - U0)) < 1e-10
    assert np.max(np.abs(-lat.unpack_momenta(P).cpu().numpy() - P0)) < 1e-9
    lat.close()


def test_dH_scaling_gpu(U0):
    P0 = synth.gaussian_momenta(256, 102)
    etas = [synth.gaussian_spinor(128, 40 + j) for j in range(3)]
    dH = []
    mults = [4, 8, 16]
    for m in mults:
        lat = make_lattice(U0)
        sp = gpu_spec(lat, steps=(m, 2 * m, 4 * m, 8 * m), tol=1e-13, exact_start=True)
        st = lat.trajectory(sp, lat.pack_momenta(P0), [lat.pack_spinor(e) for e in etas], 0.0)
        dH.append(abs(st["dH"]))
        lat.close()
    slope = np.polyfit(np.log([1.0 / m for m in mults]), np.log(dH), 1)[0]
    print("dH", dH, "slope", slope)
    assert abs(slope - 2) < 0.15


def test_dH_scaling_non_nested_gpu(U0):
    """dH ~ h^2 also when no step size divides another: base steps (ratio, correction,
    filter, gauge) = (3, 5, 7, 11) scaled by m (the generalized merge of App. B)."""
    P0 = synth.gaussian_momenta(256, 103)
    etas = [synth.gaussian_spinor(128, 50 + j) for j in range(3)]
    dH = []
    mults = [2, 4, 8]
    for m in mults:
        lat = make_lattice(U0)
        sp = gpu_spec(lat, steps=(3 * m, 5 * m, 7 * m, 11 * m), tol=1e-13, exact_start=True)
        st = lat.trajectory(sp, lat.pack_momenta(P0), [lat.pack_spinor(e) for e in etas], 0.0)
        dH.append(abs(st["dH"]))
        lat.close()
    slope = np.polyfit(np.log([1.0 / m for m in mults]), np.log(dH), 1)[0]
    print("non-nested dH", dH, "slope", slope)
    assert abs(slope - 2) < 0.15


def test_exp_minus_dH_average_gpu(U0):
    """<exp(-dH)> = 1 within 3 sigma over a Markov chain of 120 trajectories."""
    lat = make_lattice(U0)
    sp = gpu_spec(lat, steps=(2, 3, 6, 12), tol=1e-10, exact_start=False)
    vals, acc = [], 0
    for k in range(120):
        P = lat.pack_momenta(synth.gaussian_momenta(256, 1000 + k))
        etas = [lat.pack_spinor(synth.gaussian_spinor(128, 3000 + 3 * k + j)) for j in range(3)]
        st = lat.trajectory(sp, P, etas, synth.uniform(5000 + k)[0])
        vals.append(math.exp(-st["dH"]))
        acc += st["accept"]
    m, err = np.mean(vals), np.std(vals) / math.sqrt(len(vals))
    print("<exp(-dH)> = %.4f +- %.4f, acceptance %.2f" % (m, err, acc / len(vals)))
    assert abs(m - 1) < 3 * err + 1e-3
    lat.close()


def _run(lat_U, sp_kw, P0, etas, u):
    lat = make_lattice(lat_U)
    terms = [dict(kind="ratio", op=1, op2=0, steps=6), dict(kind="heavy", op=1, steps=6),
             dict(kind="poly", op=1, n=4, mu=1.2, nu=0.9, steps=12)]
    sp = lat.spec(BETA, terms, 24, det_op=0, tol=1e-12, exact_start=True, **sp_kw)
    st = lat.trajectory(sp, lat.pack_momenta(P0), [lat.pack_spinor(e) for e in etas], u)
    Ug = lat.get_gauge().cpu().numpy()
    lat.close()
    return st, Ug


def test_batched_and_mixed_solves_in_trajectory(U0):
    """The ratio and heavy solves due at the same merged step as one multi-RHS solve
    give the FP64 single-RHS trajectory up to the solver tolerance.  The FP32 / FP16
    modes (inner solves with FP64 reliable updates to the same residual, filter-term
    force chains in FP32) give it up to the FP32 rounding of that force; their
    actions, dH and accept stay FP64."""
    from paper_1609_02652_amd.pfmp import F32, F16
    P0 = synth.gaussian_momenta(256, 103)
    etas = [synth.gaussian_spinor(128, 50 + j) for j in range(3)]
    ref, Uref = _run(U0, {}, P0, etas, 0.0)
    # FP32 filter forces (relative error ~1e-7) move the end point by ~1e-8 in the links
    # and dH, a difference of Hamiltonians of size ~1e3 here, by a few 1e-6
    for kw, tol_dh, tol_u in ((dict(batch=True), 0.0, 0.0), (dict(solver_prec=F32), 2e-5, 1e-6),
                              (dict(solver_prec=F16), 2e-5, 1e-6), (dict(solver_prec=F16, batch=True), 2e-5, 1e-6)):
        st, Ug = _run(U0, kw, P0, etas, 0.0)
        du = np.max(np.abs(Ug - Uref))
        print(kw, "dH %.12f vs %.12f, iters %d vs %d, max |dU| %.2e" % (st["dH"], ref["dH"], st["solver_iters"],
                                                                      ref["solver_iters"], du), flush=True)
        # batched FP64 solves give each right-hand side the single-RHS bits: the same trajectory
        assert abs(st["dH"] - ref["dH"]) <= tol_dh
        assert du <= tol_u


def test_trajectory_det_on_own_scale_matches_oracle(U0):
    """S_det on its own 2MN scale (one more row of the merged schedule)."""
    P0 = synth.gaussian_momenta(256, 104)
    etas = [synth.gaussian_spinor(128, 60 + j) for j in range(2)]
    ospec = oracle_spec(steps=(10, 20, 40, 80), terms=(0, 2))
    ospec["det_steps"] = 20
    ref = hmc.trajectory(ospec, U0, P0, etas, u=0.5, tol=1e-12)
    lat = make_lattice(U0)
    n_jk, n_corr, n_p, n_g = 10, 20, 40, 80
    terms = [dict(kind="poly", op=1, n=4, mu=1.2, nu=0.9, steps=n_p), dict(kind="ratio", op=1, op2=0, steps=n_jk)]
    sp = lat.spec(BETA, terms, n_g, det_op=0, tol=1e-12, exact_start=True, det_steps=20)
    st = lat.trajectory(sp, lat.pack_momenta(P0), [lat.pack_spinor(e) for e in etas], 0.5)
    print("det scale: dH gpu %.12f oracle %.12f" % (st["dH"], ref["dH"]), st["nforce"], st["nforce_det"],
          ref["nforce"], flush=True)
    assert st["nforce"] + [st["nforce_det"]] == ref["nforce"]
    assert abs(st["dH"] - ref["dH"]) < 1e-10
    lat.close()


def test_gauge_step_graphs_match_launches(U0):
    """Runs of gauge-only merged steps replayed as HIP graphs (S_det on its own scale, so
    the finest scale carries the gauge force alone) give the trajectory of the same
    launches issued one by one, bit for bit, over two trajectories in a row."""
    P0 = synth.gaussian_momenta(256, 105)
    etas = [synth.gaussian_spinor(128, 70 + j) for j in range(2)]
    terms = [dict(kind="poly", op=1, n=4, mu=1.2, nu=0.9, steps=10), dict(kind="ratio", op=1, op2=0, steps=5)]
    res = []
    for graphs in (True, False):
        lat = make_lattice(U0)
        lat.graphs(graphs)
        sp = lat.spec(BETA, terms, 40, det_op=0, tol=1e-12, exact_start=True, det_steps=10)
        out = []
        for rep in range(2):
            st = lat.trajectory(sp, lat.pack_momenta(P0), [lat.pack_spinor(e) for e in etas], 0.0)
            out.append((st["dH"], st["nforce"], lat.get_gauge().cpu().numpy()))
        lat.close()
        res.append(out)
    for (dh_g, nf_g, U_g), (dh_l, nf_l, U_l) in zip(*res):
        print("graphs dH %.15f, launches dH %.15f, nforce %s" % (dh_g, dh_l, nf_g), flush=True)
        assert dh_g == dh_l and nf_g == nf_l
        assert np.array_equal(U_g, U_l)


# The paper's other actions over the same terms (Sec. 2.2 eq. hasenbusch, 1poly, 2poly;
# Sec. 3 2MP, 1PF-2MP, 2PF-1MP), one trajectory each against the oracle.  Slots: 0 = K
# (kappa 0.120), 1 = J / J_2 (0.110), 2 = J_1 (0.100).  2-filter actions factor P_8 by
# P_2 ((2 + 1) divides (8 + 1)); few 2MN steps keep the oracle's trajectory short.
KAPPA_1 = 0.100
KAPPAS = {0: KAPPA, 1: KAPPA_H, 2: KAPPA_1}


def _poly(kind, op, n, steps, n1=0):
    return dict(kind=kind, op=op, n=n, n1=n1, mu=1.2, nu=0.9, steps=steps)


ZOO = {
    "1MP": [dict(kind="heavy", op=1, steps=4), dict(kind="ratio", op=1, op2=0, steps=3)],
    "2MP": [dict(kind="heavy", op=2, steps=4), dict(kind="ratio", op=2, op2=1, steps=3),
            dict(kind="ratio", op=1, op2=0, steps=3)],
    "1PF": [_poly("poly", 0, 4, 6), _poly("polycorr", 0, 4, 3)],
    "2PF": [_poly("poly", 0, 2, 8), _poly("polyq", 0, 8, 4, n1=2), _poly("polycorr", 0, 8, 3)],
    "2PF-1MP": [_poly("poly", 1, 2, 8), _poly("polyq", 1, 8, 4, n1=2), _poly("polycorr", 1, 8, 4),
                dict(kind="ratio", op=1, op2=0, steps=3)],
    "1PF-2MP": [_poly("poly", 2, 4, 6), _poly("polycorr", 2, 4, 4), dict(kind="ratio", op=2, op2=1, steps=3),
                dict(kind="ratio", op=1, op2=0, steps=3)],
}


def _oracle_term(t):
    o = {k: v for k, v in t.items() if k not in ("op", "op2")}
    if t["kind"] == "ratio":
        o["kappa_num"], o["kappa_den"] = KAPPAS[t["op"]], KAPPAS[t["op2"]]
    else:
        o["kappa"] = KAPPAS[t["op"]]
    return o


@pytest.mark.parametrize("name", list(ZOO))
def test_action_variants_match_oracle(U0, name):
    """One trajectory of each action (heatbath, H, 2MN MD with the generalized merge, the
    accept) on 4^4 against the oracle, CG 1e-12: H0, dH, accept, links and momenta."""
    print("action variant", name, flush=True)
    terms = ZOO[name]
    P0 = synth.gaussian_momenta(256, 300)
    etas = [synth.gaussian_spinor(128, 310 + j) for j in range(len(terms))]
    u = synth.uniform(326)[0]   # 0.048: accepted, so the final links are compared too
    ospec = dict(dims=DIMS, beta=BETA, csw=CSW, kappa=KAPPA, gauge_steps=16,
                 terms=[_oracle_term(t) for t in terms])
    ref = hmc.trajectory(ospec, U0, P0, etas, u=u, tol=1e-12)
    lat = make_lattice(U0)
    lat.set_operator(2, KAPPA_1, CSW)
    sp = lat.spec(BETA, terms, 16, det_op=0, tol=1e-12, exact_start=True)
    Pend = lat.pack_momenta(np.zeros((256, 4, 8)))
    st = lat.trajectory(sp, lat.pack_momenta(P0), [lat.pack_spinor(e) for e in etas], u, P_end=Pend)
    print("dH gpu %.12f oracle %.12f" % (st["dH"], ref["dH"]), st["nforce"], ref["nforce"], flush=True)
    assert list(st["nforce"][:len(terms) + 1]) == list(ref["nforce"])
    assert abs(st["H0"] - ref["H0"]) < 1e-8 * abs(ref["H0"])
    Ug = lat.get_gauge().cpu().numpy()
    Pg = lat.unpack_momenta(Pend).cpu().numpy()
    print("|dH - dH_oracle| %.2e, max |U - U_oracle| %.2e, max |P - P_oracle| %.2e"
          % (abs(st["dH"] - ref["dH"]), np.max(np.abs(Ug - ref["U"])), np.max(np.abs(Pg - ref["P"]))), flush=True)
    assert abs(st["dH"] - ref["dH"]) < 1e-10
    assert st["accept"] == ref["accept"]
    if st["accept"]:
        assert np.max(np.abs(Ug - ref["U"])) < 1e-10
    else:
        assert np.array_equal(Ug, U0)
    assert np.max(np.abs(lat.unpack_momenta(Pend).cpu().numpy() - ref["P"])) < 1e-8
    lat.close()


def test_step_tuner_on_gpu(U0):
    """The tuner's loop over the library (Sec. 2.4): measured maximal forces per row, steps
    with F_i h_i = c, rounds of trajectories rescaling c; the gauge force is the largest, and
    each round's steps keep every row at or below c."""
    from paper_1609_02652_amd import tuner
    lat = make_lattice(U0)

    def build(steps):
        n_g, n_p, n_c, n_r = steps[:4]
        return gpu_spec(lat, steps=(n_r, n_c, n_p, n_g), tol=1e-10, exact_start=False)
    T = tuner.StepTuner(lat, build, 3)
    F = T.measure_forces([80, 40, 20, 10, 1], 2)
    print("forces", F.tolist(), flush=True)
    assert F.shape == (5, 2) and np.all(F[:, 0] > 0) and np.all(F[:, 0] >= F[:, 1])
    assert F[0, 0] == F[:, 0].max()
    fmax = list(F[:4, 0])
    hist, best = T.tune(fmax, c0=fmax[3] / 10, ntraj=2, rounds=2)
    assert 0 <= best < len(hist)
    for c, steps, traj in hist:
        assert all(f / n <= c * (1 + 1e-12) for f, n in zip(fmax, steps))
        assert all(math.isfinite(t[0]) and t[2] > 0 for t in traj)
        print("c %.4f steps %s dH %s" % (c, steps, [round(t[0], 4) for t in traj]), flush=True)
    lat.close()


def test_trajectory_failure_restores_start_field():
    """A trajectory whose solve hits maxiter after the links have moved returns NOCONV
    and leaves the context on its start field: free field U = 1 (Wilson, kappa 0.12), one
    heavy term with phi = W^dag eta for a plane wave eta chosen as an eigenvector of Khat,
    so the solve of the first force step converges in one CG iteration (maxiter = 1);
    after the first link update the field is no longer free, the next solve stops at
    maxiter, and the links must come back bit for bit.  A trajectory run afterwards on the
    same context must give the bits of one on a fresh context."""
    from paper_1609_02652_amd.pfmp import Lattice, PfmpError
    U1 = synth.unit_gauge(DIMS)
    n = (1, 0, 0, 0)
    p = [2 * math.pi * n[m] / DIMS[m] for m in range(3)] + [2 * math.pi * (n[3] + 0.5) / DIMS[3]]
    b = [2 * math.sin(q) for q in p]
    bg = sum(b[m] * oracle.gamma(m) for m in range(4))
    w, v = np.linalg.eigh(bg)
    u = np.outer(v[:, 0], [1.0, 0.3j, -0.2])
    lexeo, _, _ = oracle.index_maps(DIMS)
    eta = np.zeros((len(lexeo[0]), 4, 3), np.complex128)
    for i, x in enumerate(lexeo[0]):
        c, r = [], int(x)
        for L in DIMS:
            c.append(r % L)
            r //= L
        eta[i] = np.exp(1j * sum(p[m] * c[m] for m in range(4))) * u
    P0 = synth.gaussian_momenta(256, 107)

    def lattice():
        lat = Lattice(DIMS)
        lat.set_gauge(U1)
        lat.set_operator(0, 0.12, 0.0)
        return lat

    terms = [dict(kind="heavy", op=0, steps=1)]
    lat = lattice()
    sp = lat.spec(BETA, terms, 2, det_op=-1, tol=1e-12, maxiter=1, exact_start=False)
    with pytest.raises(PfmpError) as e:
        lat.trajectory(sp, lat.pack_momenta(P0), [lat.pack_spinor(eta)], 0.5)
    assert e.value.code == -3
    assert np.array_equal(lat.get_gauge().cpu().numpy(), U1)
    # the same trajectory with room to converge, here and on a fresh context
    sp2 = lat.spec(BETA, terms, 2, det_op=-1, tol=1e-12, maxiter=10000, exact_start=False)
    st = lat.trajectory(sp2, lat.pack_momenta(P0), [lat.pack_spinor(eta)], 0.0)
    U_here = lat.get_gauge().cpu().numpy()
    lat.close()
    fresh = lattice()
    st2 = fresh.trajectory(fresh.spec(BETA, terms, 2, det_op=-1, tol=1e-12, maxiter=10000, exact_start=False),
                           fresh.pack_momenta(P0), [fresh.pack_spinor(eta)], 0.0)
    print("after the failure: dH %.12f, fresh context %.12f" % (st["dH"], st2["dH"]), flush=True)
    assert st["dH"] == st2["dH"] and st["accept"] == 1
    assert np.array_equal(U_here, fresh.get_gauge().cpu().numpy())
    assert not np.array_equal(U_here, U1)
    fresh.close()


# The structure of the light-quark trajectory workload (48^3 x 96): a three-level filter nest
# on the heaviest J (P_2, Q = P_8 / P_2, Q = P_26 / P_8 and the correction [J P_26(J)]^-1; the
# degrees of the workload's nest (6, 20, 62) scaled down with the same divisibility), three
# Hasenbusch ratios down to the target K, S_det, and four integrator scales, on 4^4 against
# the oracle.  Slots: 0 = K (0.120), 1 = 0.110, 2 = 0.100, 3 = 0.090 (the heaviest J).
NEST_KAPPAS = {0: 0.120, 1: 0.110, 2: 0.100, 3: 0.090}
NEST = [_poly("poly", 3, 2, 6), _poly("polyq", 3, 8, 6, n1=2), _poly("polyq", 3, 26, 6, n1=8),
        _poly("polycorr", 3, 26, 4), dict(kind="ratio", op=3, op2=2, steps=4),
        dict(kind="ratio", op=2, op2=1, steps=3), dict(kind="ratio", op=1, op2=0, steps=3)]


def _nest_oracle_term(t):
    o = {k: v for k, v in t.items() if k not in ("op", "op2")}
    if t["kind"] == "ratio":
        o["kappa_num"], o["kappa_den"] = NEST_KAPPAS[t["op"]], NEST_KAPPAS[t["op2"]]
    else:
        o["kappa"] = NEST_KAPPAS[t["op"]]
    return o


def _nest_lattice(U0):
    lat = make_lattice(U0)
    lat.set_operator(1, NEST_KAPPAS[1], CSW)
    lat.set_operator(2, NEST_KAPPAS[2], CSW)
    lat.set_operator(3, NEST_KAPPAS[3], CSW)
    return lat


def test_filter_nest_with_three_ratios_matches_oracle(U0):
    """One trajectory of the three-level filter nest with three Hasenbusch ratios and four
    integrator scales: H0, dH, accept, force counts, links and momenta against the oracle."""
    P0 = synth.gaussian_momenta(256, 500)
    etas = [synth.gaussian_spinor(128, 510 + j) for j in range(len(NEST))]
    ospec = dict(dims=DIMS, beta=BETA, csw=CSW, kappa=NEST_KAPPAS[0], gauge_steps=12,
                 terms=[_nest_oracle_term(t) for t in NEST])
    ref = hmc.trajectory(ospec, U0, P0, etas, u=0.3, tol=1e-12)
    lat = _nest_lattice(U0)
    sp = lat.spec(BETA, NEST, 12, det_op=0, tol=1e-12, exact_start=True)
    Pend = lat.pack_momenta(np.zeros((256, 4, 8)))
    st = lat.trajectory(sp, lat.pack_momenta(P0), [lat.pack_spinor(e) for e in etas], 0.3, P_end=Pend)
    Ug = lat.get_gauge().cpu().numpy()
    Pg = lat.unpack_momenta(Pend).cpu().numpy()
    print("nest: dH gpu %.12f oracle %.12f, max |dU| %.2e, max |dP| %.2e" % (
        st["dH"], ref["dH"], np.max(np.abs(Ug - ref["U"])), np.max(np.abs(Pg - ref["P"]))), flush=True)
    assert list(st["nforce"][:len(NEST) + 1]) == list(ref["nforce"])
    assert abs(st["H0"] - ref["H0"]) < 1e-8 * abs(ref["H0"])
    assert abs(st["dH"] - ref["dH"]) < 1e-10
    assert st["accept"] == ref["accept"]
    if st["accept"]:
        assert np.max(np.abs(Ug - ref["U"])) < 1e-10
    assert np.max(np.abs(Pg - ref["P"])) < 1e-8
    lat.close()


def test_filter_nest_mixed_modes_track_fp64(U0):
    """The same nest in the chosen mixed-precision modes (FP16-storage and FP32 inner CG with
    FP64 reliable updates, FP32 filter-force chains; actions and the accept in FP64) and with
    batched ratio solves: dH within the FP32 force rounding of the FP64 trajectory."""
    from paper_1609_02652_amd.pfmp import F32, F16
    P0 = synth.gaussian_momenta(256, 501)
    etas = [synth.gaussian_spinor(128, 520 + j) for j in range(len(NEST))]
    res = {}
    for name, kw in (("f64", {}), ("f32", dict(solver_prec=F32)), ("f16", dict(solver_prec=F16)),
                     ("f64_batch", dict(batch=True)), ("f16_batch", dict(solver_prec=F16, batch=True))):
        lat = _nest_lattice(U0)
        sp = lat.spec(BETA, NEST, 12, det_op=0, tol=1e-12, exact_start=True, **kw)
        st = lat.trajectory(sp, lat.pack_momenta(P0), [lat.pack_spinor(e) for e in etas], 0.0)
        res[name] = (st["dH"], lat.get_gauge().cpu().numpy())
        print("nest %s: dH %.12f, iters %d" % (name, st["dH"], st["solver_iters"]), flush=True)
        lat.close()
    dh0, U64 = res["f64"]
    assert res["f64_batch"][0] == dh0 and np.array_equal(res["f64_batch"][1], U64)
    for name in ("f32", "f16", "f16_batch"):
        assert abs(res[name][0] - dh0) < 2e-5
        assert np.max(np.abs(res[name][1] - U64)) < 1e-6
