// solver.hip -- CG on Khat and multi-shift CG (paper Sec. 2.1; App. C), FP64.
//
// The iteration never waits for the host: every scalar (alpha, beta, |r|^2, the
// shift recurrences) lives in device memory and is formed from block partials in one
// fixed order (partials_total): by every block of the kernel that needs it while the
// lattice gives few partials, else once by a one-block kernel.  A "done" flag written
// on the device turns the remaining launches of a chunk into early exits; the host only
// looks at it once per chunk of iterations.
//
// CG iteration (5 launches, 7 on large lattices): hop1, hop2 (|Mhat p|^2 = <p, Khat p>
// partials), [its total], hop3, hop4 fused with alpha, x += alpha p, r -= alpha Khat p and
// the |r+|^2 partials, [|r+|^2, beta and the stop test], p = r + beta p.
#include <chrono>
#include <cmath>
#include <vector>

#include "hop.h"

namespace {

// device scalar slots in ctx->scal
enum { S_RR = 0, S_THR, S_PAP, S_ALPHA, S_BETA, S_ITER, S_DONE, S_MAXIT, S_BB, S_APREV, S_BPREV, S_CACT, S_NACT,
       S_RROLD,     // |r|^2 at the start of the iteration (stage 4, for beta)
       S_ITNEXT };  // iteration count after this iteration (stage 4, for the stop decision)
constexpr int kShiftBase = 64;   // per-shift records start here
struct ShiftRec {                // 16 doubles
    double2 sigma, zp, z, zn, as, bs;
    double active, upd, res2, pad;
};

__device__ __forceinline__ double2 cdiv(double2 a, double2 b)
{
    double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// zeta_{k+1} and alpha_s of every active shift from the base alpha (Jegerlehner's
// recurrences), one thread per shift; called by one block only
__device__ __forceinline__ void ms_shift_alphas(double alpha, const double *__restrict__ st, int ns,
                                                ShiftRec *__restrict__ rec)
{
    const double ap = st[S_APREV], bp = st[S_BPREV];
    for (int s = threadIdx.x; s < ns; s += blockDim.x) {
        ShiftRec q = rec[s];
        if (q.active == 0) continue;
        // zn = z zp ap / (alpha bp (zp - z) + zp ap (1 + sigma alpha))
        double2 num = cscale(cmul(q.z, q.zp), ap);
        double2 one_sa = make_double2(1 + q.sigma.x * alpha, q.sigma.y * alpha);
        double2 den = cadd(cscale(csub(q.zp, q.z), alpha * bp), cscale(cmul(q.zp, one_sa), ap));
        q.zn = cdiv(num, den);
        q.as = cscale(cdiv(q.zn, q.z), alpha);
        rec[s] = q;
    }
}

__global__ void k_cg_init(const double *__restrict__ partials, int nparts, double tol2, int maxiter,
                          double *__restrict__ st)
{
    __shared__ double sh[kRedBlock / 64];
    double s = 0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) s += partials[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double bb = 0;
        for (int k = 0; k < kRedBlock / 64; k++) bb += sh[k];
        st[S_RR] = bb;
        st[S_BB] = bb;
        st[S_THR] = tol2 * bb;
        st[S_ITER] = 0;
        st[S_DONE] = bb == 0 ? 1 : 0;
        st[S_MAXIT] = maxiter;
        st[S_APREV] = 1;
        st[S_BPREV] = 0;
        st[S_CACT] = 0;
    }
}

// Khat p from t = Mhat p and T' = A_oo^-1 D_oe g5 t:  Kp = g5 (A_ee g5 t - kappa^2 D_eo T');
// then x += alpha p, r -= alpha Kp and the |r+|^2 partials.  alpha = |r|^2 / <p, Khat p>:
// INL = 1, every block forms <p, Khat p> from the stage-2 partials (part_pap, npap), and
// block 0 records it with alpha, |r|^2 (S_RROLD) and the next iteration count (S_ITNEXT)
// for the p update; INL = 0, <p, Khat p> was totalled into S_PAP by a one-block kernel.
// MS (multi-shift): block 0 also steps the shifts' zeta and alpha_s.
template <int CLOV, int LM, int MS, int INL>
__global__ __launch_bounds__(kBlock) void k_cg_hop4(Geom g, const double2 *__restrict__ t,
                                                    const double2 *__restrict__ T, const double2 *__restrict__ U,
                                                    const double *__restrict__ cl, double a,
                                                    const double2 *__restrict__ p, double2 *__restrict__ x,
                                                    double2 *__restrict__ r, double *__restrict__ st,
                                                    double *__restrict__ partials, const double *__restrict__ part_pap,
                                                    int npap, ShiftRec *__restrict__ rec = nullptr, int ns = 0)
{
    if (st[S_DONE] != 0) return;
    double pap;
    if (INL) {
        double tp[1];
        partials_total<kBlock, 1, kInlineChunks>(part_pap, npap, tp);
        pap = tp[0];
    } else {
        pap = st[S_PAP];
    }
    const double alpha = st[S_RR] / pap;
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            st[S_ALPHA] = alpha;
            if (INL) {
                st[S_PAP] = pap;
                st[S_RROLD] = st[S_RR];
                st[S_ITNEXT] = st[S_ITER] + 1;
            }
        }
        if (MS) ms_shift_alphas(alpha, st, ns, rec);
    }
    const int tt = xcd_site(2 * g.Vh);
    double nrm = 0;
    if (tt >= 0) {
        const int i = tile_site(g, tt >> 1), hb = tt & 1;
        double2 acc[6], tv[6], at[6];
        hop_pair<LM, double2>(g, 0, i, hb, T, U, 1.0, acc);
        // site-local vectors: non-temporal when the links stream (large lattices)
        constexpr int ST = (LM >> 1) & 1;
        load_block_st<ST>(t, g.Vh, i, hb, -1.0, tv);
        if (CLOV) clover_block<double, double2>(cl, g.Vh, i, hb, tv, at);
        const long Vh = g.Vh;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            double2 base = CLOV ? at[k] : tv[k];
            double2 kp = make_double2(fmadd(a, acc[k].x, base.x), fmadd(a, acc[k].y, base.y));
            if (hb) kp = cneg(kp);
            const long e = (long)(6 * hb + k) * Vh + i;
            double2 pv = ld_st<ST>(p + e), xv = ld_st<ST>(x + e), rv = ld_st<ST>(r + e);
            xv.x = fmadd(alpha, pv.x, xv.x); xv.y = fmadd(alpha, pv.y, xv.y);
            rv.x = fmadd(-alpha, kp.x, rv.x); rv.y = fmadd(-alpha, kp.y, rv.y);
            st_st<ST>(x + e, xv);
            st_st<ST>(r + e, rv);
            cnorm_acc(nrm, rv);
        }
    }
    const double v[1] = {nrm};
    op_partials_store<kBlock, 1>(v, partials);
}

// stage 4 of the fused CG (with rec: of the multi-shift CG)
static void launch_cg_hop4(pfmp_ctx *ctx, bool cl, bool inl, int nb, const double2 *t, const double2 *T,
                           const double *clov, double mk2, const double2 *p, double2 *x, double2 *r, double *part,
                           const double *part_pap, ShiftRec *rec = nullptr, int ns = 0)
{
#define HOP4(CL, LM, MS, IN)                                                                                     \
    hipLaunchKernelGGL((k_cg_hop4<CL, LM, MS, IN>), dim3(nb), dim3(kBlock), 0, ctx->stream, ctx->g, t, T, ctx->U, \
                       clov, mk2, p, x, r, ctx->scal, part, part_pap, nb, rec, ns)
#define HOP4_11(LM) if (inl) HOP4(1, LM, 1, 1); else HOP4(1, LM, 1, 0)
#define HOP4_10(LM) if (inl) HOP4(1, LM, 0, 1); else HOP4(1, LM, 0, 0)
#define HOP4_01(LM) if (inl) HOP4(0, LM, 1, 1); else HOP4(0, LM, 1, 0)
#define HOP4_00(LM) if (inl) HOP4(0, LM, 0, 1); else HOP4(0, LM, 0, 0)
    const int lm = link_mode(ctx->g);
    if (cl && rec) { PFMP_LM_SWITCH(lm, HOP4_11) }
    else if (cl) { PFMP_LM_SWITCH(lm, HOP4_10) }
    else if (rec) { PFMP_LM_SWITCH(lm, HOP4_01) }
    else { PFMP_LM_SWITCH(lm, HOP4_00) }
#undef HOP4_11
#undef HOP4_10
#undef HOP4_01
#undef HOP4_00
#undef HOP4
}

// |r+|^2 from the stage-4 partials, beta = |r+|^2 / |r|^2 and the stop decision; one
// workgroup (many partials)
__global__ __launch_bounds__(kFinishThreads) void k_cg_finish_rr(const double *__restrict__ part, int n,
                                                                double *__restrict__ st)
{
    if (st[S_DONE] != 0) return;
    double t[1];
    partials_total<kFinishThreads, 1, kMaxChunks>(part, n, t);
    if (threadIdx.x == 0) {
        const double rr = t[0], it = st[S_ITER] + 1;
        st[S_BETA] = rr / st[S_RR];
        st[S_RR] = rr;
        st[S_ITER] = it;
        st[S_DONE] = rr <= st[S_THR] ? 1 : (it >= st[S_MAXIT] ? 2 : 0);
    }
}

// p = r + beta p.  INL = 1: every block forms |r+|^2 from the stage-4 partials and with it
// beta = |r+|^2 / S_RROLD and the stop decision (iteration count S_ITNEXT, written by stage
// 4), all the same in every block; block 0 records them.  (A block that starts after block 0
// has written S_DONE returns at once, as it would have after taking the same decision.)
// INL = 0: beta and the decision were recorded by k_cg_finish_rr.
template <int INL>
__global__ __launch_bounds__(kRedBlock) void k_cg_update_p(long n, const double2 *__restrict__ r,
                                                           double2 *__restrict__ p, double *__restrict__ st,
                                                           const double *__restrict__ part_rr, int nrr)
{
    if (st[S_DONE] != 0) return;
    double b;
    if (INL) {
        double tr[1];
        partials_total<kRedBlock, 1, kInlineChunks>(part_rr, nrr, tr);
        const double rr = tr[0], it = st[S_ITNEXT];
        const int done = rr <= st[S_THR] ? 1 : (it >= st[S_MAXIT] ? 2 : 0);
        b = rr / st[S_RROLD];
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st[S_BETA] = b;
            st[S_RR] = rr;
            st[S_ITER] = it;
            st[S_DONE] = done;
        }
        if (done) return;
    } else {
        b = st[S_BETA];
    }
    // six complex numbers per lane (grid-stride), so that a sixth as many workgroups form the
    // inline total
    const long stride = (long)gridDim.x * blockDim.x;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += stride) {
        double2 rv = r[e], pv = p[e];
        p[e] = make_double2(fmadd(b, pv.x, rv.x), fmadd(b, pv.y, rv.y));
    }
}


__global__ void k_residual(long n, const double2 *__restrict__ b, const double2 *__restrict__ Ax, double2 zr,
                           const double2 *__restrict__ x, double2 *__restrict__ r)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    // r = b - (A x - z x)
    double2 v = csub(Ax[t], cmul(zr, x[t]));
    r[t] = csub(b[t], v);
}

// ---------------------------------------------------------------- multi-shift



__global__ void k_ms_init(int ns, const double *__restrict__ zs, ShiftRec *__restrict__ rec)
{
    int s = threadIdx.x;
    if (s >= ns) return;
    ShiftRec q;
    q.sigma = make_double2(-zs[2 * s], -zs[2 * s + 1]);   // (Khat + sigma), sigma = -z
    q.zp = q.z = q.zn = make_double2(1, 0);
    q.as = q.bs = make_double2(0, 0);
    q.active = 1;
    q.upd = 0;
    q.res2 = 0;
    q.pad = 0;
    rec[s] = q;
}

__global__ __launch_bounds__(kFinishThreads) void k_ms_beta(const double *__restrict__ partials, int nparts,
                                                            int ns, double *__restrict__ st,
                                                            ShiftRec *__restrict__ rec)
{
    if (st[S_DONE] != 0) {
        if (threadIdx.x == 0) st[S_CACT] = 0;
        return;
    }
    double tr[1];
    partials_total<kFinishThreads, 1, kMaxChunks>(partials, nparts, tr);
    const double rr = tr[0];
    double beta = rr / st[S_RR];
    __shared__ int nact;
    if (threadIdx.x == 0) nact = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < ns; s += blockDim.x) {
        ShiftRec q = rec[s];
        q.upd = q.active;
        if (q.active != 0) {
            double2 ratio = cdiv(q.zn, q.z);
            q.bs = cscale(cmul(ratio, ratio), beta);
            q.res2 = (q.zn.x * q.zn.x + q.zn.y * q.zn.y) * rr;
            q.zp = q.z;
            q.z = q.zn;
            if (q.res2 <= st[S_THR]) q.active = 0;
            else atomicAdd(&nact, 1);
        }
        rec[s] = q;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st[S_APREV] = st[S_ALPHA];
        st[S_BPREV] = beta;
        st[S_BETA] = beta;
        st[S_RR] = rr;
        st[S_ITER] += 1;
        st[S_NACT] = nact;
        st[S_CACT] = 1;
        st[S_DONE] = nact == 0 ? 1 : (st[S_ITER] >= st[S_MAXIT] ? 2 : 0);
    }
}

// x_s += alpha_s p_s; p_s = zeta_{k+1} r + beta_s p_s (shifts updated this step); p = r + beta p
__global__ __launch_bounds__(256) void k_ms_update(long n, int ns, const double2 *__restrict__ r,
                                                   double2 *__restrict__ p, double2 *const *__restrict__ xs,
                                                   double2 *const *__restrict__ ps,
                                                   const ShiftRec *__restrict__ rec, const double *__restrict__ st)
{
    if (st[S_CACT] == 0) return;
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    double2 rv = r[t];
    for (int s = 0; s < ns; s++) {
        if (rec[s].upd == 0) continue;
        double2 as = rec[s].as, bs = rec[s].bs, zn = rec[s].zn;
        double2 pv = ps[s][t];
        double2 xv = xs[s][t];
        cfma(xv, as, pv);
        xs[s][t] = xv;
        double2 np = cmul(zn, rv);
        cfma(np, bs, pv);
        ps[s][t] = np;
    }
    double b = st[S_BETA];
    double2 pv = p[t];
    p[t] = make_double2(rv.x + b * pv.x, rv.y + b * pv.y);
}

}  // namespace

// ---------------------------------------------------------------- host drivers

static int check_solver_args(pfmp_ctx *ctx, int op, const pfmp_solver_params *p)
{
    if (!ctx) return PFMP_ERR_ARG;
    if (op < 0 || op >= PFMP_MAX_OPS) return set_err(ctx, PFMP_ERR_ARG, "operator slot out of range");
    if (!ctx->have_gauge || !ctx->ops[op].valid) return set_err(ctx, PFMP_ERR_STATE, "operator not configured");
    if (!p || !(p->tol > 0) || p->maxiter <= 0) return set_err(ctx, PFMP_ERR_ARG, "solver parameters");
    int rc = op_ready(ctx, op);
    return rc ? rc : gauge_f32_ready(ctx);
}

struct CGBufs {
    double2 *r, *p, *t, *T, *Kx;
    double *part_a, *part_b;
};

static int cg_bufs(pfmp_ctx *ctx, CGBufs &B)
{
    size_t vb = sizeof(double) * spinor_reals(ctx->g);
    size_t pb = sizeof(double) * (op_nparts(ctx->g) + 64);
    B.r = (double2 *)ws_alloc(ctx, vb, 4);
    B.p = (double2 *)ws_alloc(ctx, vb, 5);
    B.t = (double2 *)ws_alloc(ctx, vb, 6);
    B.T = (double2 *)ws_alloc(ctx, vb, 7);
    B.Kx = (double2 *)ws_alloc(ctx, vb, 8);
    B.part_a = (double *)ws_alloc(ctx, pb, 9);
    B.part_b = (double *)ws_alloc(ctx, pb, 10);
    if (!B.r || !B.p || !B.t || !B.T || !B.Kx || !B.part_a || !B.part_b)
        return set_err(ctx, PFMP_ERR_OOM, "solver workspace");
    return 0;
}

// |b - (Khat - z) x| / |b| in FP64 (synchronises)
static int true_residual(pfmp_ctx *ctx, int op, const double2 *b, const double2 *x, double2 z, CGBufs &B,
                         double *res)
{
    long n = 12L * ctx->g.Vh;
    int rc = op_apply_K(ctx, op, x, B.Kx, B.t, B.T, nullptr);
    if (rc) return rc;
    hipLaunchKernelGGL(k_residual, dim3(nblocks(n, 256)), dim3(256), 0, ctx->stream, n, b, B.Kx, z, x, B.r);
    LAUNCHCHK(ctx);
    double v[2];
    if ((rc = launch_norm2(ctx, B.r, n, ctx->red))) return rc;
    if ((rc = red_finish(ctx, ctx->red, ctx->nblk_red, 1, v))) return rc;
    if ((rc = launch_norm2(ctx, b, n, ctx->red))) return rc;
    if ((rc = red_finish(ctx, ctx->red, ctx->nblk_red, 1, v + 1))) return rc;
    *res = v[1] > 0 ? std::sqrt(v[0] / v[1]) : 0.0;
    return 0;
}

// Iterations to issue before the next look at the device state: the remaining count
// predicted from the residual's decay over the last chunk, plus one (4 .. 200).
static int next_chunk(double rr, double thr, double it, double rr_prev, double it_prev)
{
    if (!(rr_prev > 0) || !(rr > 0) || it <= it_prev || rr >= rr_prev) return 25;
    const double rate = std::log(rr / rr_prev) / (it - it_prev);   // log decay per iteration
    const double left = std::log(thr / rr) / rate;
    const int c = (int)std::ceil(left) + 1;
    return c < 4 ? 4 : (c > 200 ? 200 : c);
}

static int read_state(pfmp_ctx *ctx, double *h, int n)
{
    HIPCHK(ctx, hipMemcpyAsync(ctx->red_host, ctx->scal, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < n; k++) h[k] = ctx->red_host[k];
    return 0;
}

extern "C" int pfmp_cg_solve(pfmp_ctx *ctx, int op, const void *b_, void *x_, const pfmp_solver_params *prm,
                             pfmp_solver_stats *st)
{
    int rc = check_solver_args(ctx, op, prm);
    if (rc) return rc;
    if (!b_ || !x_) return set_err(ctx, PFMP_ERR_ARG, "cg_solve: null buffer");
    if (prm->prec != PFMP_F64) return cg_solve_mixed(ctx, op, b_, x_, prm, st);
    auto t0 = std::chrono::steady_clock::now();
    const Geom &g = ctx->g;
    OpSlot &s = ctx->ops[op];
    CGBufs B;
    if ((rc = cg_bufs(ctx, B))) return rc;
    const double2 *b = (const double2 *)b_;
    double2 *x = (double2 *)x_;
    long n = 12L * g.Vh;
    size_t vb = sizeof(double) * spinor_reals(g);
    int nb = op_nparts(g);
    HIPCHK(ctx, hipMemsetAsync(x, 0, vb, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(B.r, b, vb, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(B.p, b, vb, hipMemcpyDeviceToDevice, ctx->stream));
    if ((rc = launch_norm2(ctx, b, n, ctx->red))) return rc;
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(kRedBlock), 0, ctx->stream, ctx->red, ctx->nblk_red,
                       prm->tol * prm->tol, prm->maxiter, ctx->scal);
    LAUNCHCHK(ctx);
    const bool cl = s.csw != 0;
    const double mk2 = -s.kappa * s.kappa;
    const bool inl = totals_inline(nb);
    int chunk = prm->check_every > 0 ? prm->check_every : 25;
    double h[16], rr_prev = 0, it_prev = 0;
    // one iteration: 5 launches with fixed arguments (7 with the two one-block totals of a
    // large lattice), replayed as a graph
    auto iteration = [&]() -> int {
        int e;
        // t = Mhat p, with <p, Khat p> = |t|^2 partials
        if ((e = clovinv64(ctx, 1, B.p, s.clov[1], B.T, 1.0, 1.0, cl, ctx->scal + S_DONE))) return e;
        if ((e = xpay64(ctx, 0, B.p, B.T, s.clov[0], mk2, B.t, 1.0, cl, B.part_a, ctx->scal + S_DONE))) return e;
        if (!inl && (e = launch_total<1>(ctx, B.part_a, nb, ctx->scal + S_PAP, ctx->scal + S_DONE))) return e;
        // T' = A_oo^-1 D_oe g5 t
        if ((e = clovinv64(ctx, 1, B.t, s.clov[1], B.T, -1.0, 1.0, cl, ctx->scal + S_DONE))) return e;
        // alpha, x and r updates and the |r+|^2 partials; then beta, the stop test and p
        launch_cg_hop4(ctx, cl, inl, nb, B.t, B.T, s.clov[0], mk2, B.p, x, B.r, B.part_b, B.part_a);
        if (!inl)
            hipLaunchKernelGGL(k_cg_finish_rr, dim3(1), dim3(kFinishThreads), 0, ctx->stream, B.part_b, nb,
                               ctx->scal);
        if (inl)
            hipLaunchKernelGGL(k_cg_update_p<1>, dim3(nblocks((n + 5) / 6, kRedBlock)), dim3(kRedBlock), 0, ctx->stream, n,
                               B.r, B.p, ctx->scal, B.part_b, nb);
        else
            hipLaunchKernelGGL(k_cg_update_p<0>, dim3(nblocks((n + 5) / 6, kRedBlock)), dim3(kRedBlock), 0, ctx->stream, n,
                               B.r, B.p, ctx->scal, B.part_b, nb);
        LAUNCHCHK(ctx);
        return 0;
    };
    std::vector<uint64_t> key;
    key_add(key, 1);   // FP64 CG iteration
    key_geom(key, g);
    for (const void *ptr : {(const void *)B.p, (const void *)B.T, (const void *)B.t, (const void *)B.r,
                            (const void *)B.part_a, (const void *)B.part_b, (const void *)x, (const void *)ctx->U,
                            (const void *)ctx->scal, (const void *)s.clov[0], (const void *)s.clov[1]})
        key_add(key, ptr);
    key_add(key, mk2);
    key_add(key, (int)cl);
    for (;;) {
        if ((rc = graph_run(ctx, key, chunk, iteration))) return rc;
        if ((rc = read_state(ctx, h, 16))) return rc;
        if (h[S_DONE] != 0) break;
        if (prm->check_every <= 0) chunk = next_chunk(h[S_RR], h[S_THR], h[S_ITER], rr_prev, it_prev);
        rr_prev = h[S_RR];
        it_prev = h[S_ITER];
    }
    int iters = (int)h[S_ITER];
    double res = 0;
    if ((rc = true_residual(ctx, op, b, x, make_double2(0, 0), B, &res))) return rc;
    auto t1 = std::chrono::steady_clock::now();
    if (st) {
        st->iters = iters;
        st->reliable_updates = 0;
        st->true_res = res;
        st->seconds = std::chrono::duration<double>(t1 - t0).count();
        st->kmults = iters + 1;
    }
    if (h[S_DONE] == 2 && !(res <= prm->tol)) return set_err(ctx, PFMP_ERR_NOCONV, "cg_solve: maxiter reached");
    return 0;
}

extern "C" int pfmp_cg_multishift(pfmp_ctx *ctx, int op, int nshift, const double *z, const void *b_,
                                  void *const *x_, const pfmp_solver_params *prm, pfmp_solver_stats *st)
{
    int rc = check_solver_args(ctx, op, prm);
    if (rc) return rc;
    if (nshift <= 0 || nshift > PFMP_MAX_SHIFTS || !z || !b_ || !x_)
        return set_err(ctx, PFMP_ERR_ARG, "cg_multishift: bad shifts or buffers");
    for (int k = 0; k < nshift; k++)
        if (!x_[k]) return set_err(ctx, PFMP_ERR_ARG, "cg_multishift: null solution buffer");
    auto t0 = std::chrono::steady_clock::now();
    const Geom &g = ctx->g;
    OpSlot &s = ctx->ops[op];
    CGBufs B;
    if ((rc = cg_bufs(ctx, B))) return rc;
    long n = 12L * g.Vh;
    size_t vb = sizeof(double) * spinor_reals(g);
    int nb = op_nparts(g);
    double2 *pbuf = (double2 *)ws_alloc(ctx, vb * nshift, 11);
    double2 **ptrs = (double2 **)ws_alloc(ctx, sizeof(double2 *) * 2 * nshift, 12);
    double *zdev = (double *)ws_alloc(ctx, sizeof(double) * 2 * nshift, 13);
    if (!pbuf || !ptrs || !zdev) return set_err(ctx, PFMP_ERR_OOM, "multishift workspace");
    std::vector<double2 *> hp(2 * nshift);
    for (int k = 0; k < nshift; k++) {
        hp[k] = (double2 *)x_[k];
        hp[nshift + k] = pbuf + (long)k * n;
    }
    HIPCHK(ctx, hipMemcpyAsync(ptrs, hp.data(), sizeof(double2 *) * 2 * nshift, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(zdev, z, sizeof(double) * 2 * nshift, hipMemcpyHostToDevice, ctx->stream));
    const double2 *b = (const double2 *)b_;
    for (int k = 0; k < nshift; k++) {
        HIPCHK(ctx, hipMemsetAsync(x_[k], 0, vb, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(hp[nshift + k], b, vb, hipMemcpyDeviceToDevice, ctx->stream));
    }
    HIPCHK(ctx, hipMemcpyAsync(B.r, b, vb, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(B.p, b, vb, hipMemcpyDeviceToDevice, ctx->stream));
    // the base x accumulates into a scratch vector (Kx) that is not returned
    HIPCHK(ctx, hipMemsetAsync(B.Kx, 0, vb, ctx->stream));
    ShiftRec *rec = (ShiftRec *)(ctx->scal + kShiftBase);
    if ((rc = launch_norm2(ctx, b, n, ctx->red))) return rc;
    {
        double bb0 = 0;
        if ((rc = red_finish(ctx, ctx->red, ctx->nblk_red, 1, &bb0))) return rc;
        if (bb0 == 0) {   // b = 0: every x_k = 0 solves it exactly
            if (st) *st = pfmp_solver_stats{};
            return 0;
        }
    }
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(kRedBlock), 0, ctx->stream, ctx->red, ctx->nblk_red,
                       prm->tol * prm->tol, prm->maxiter, ctx->scal);
    hipLaunchKernelGGL(k_ms_init, dim3(1), dim3(PFMP_MAX_SHIFTS), 0, ctx->stream, nshift, zdev, rec);
    LAUNCHCHK(ctx);
    const bool cl = s.csw != 0;
    const double mk2 = -s.kappa * s.kappa;
    const bool inl = totals_inline(nb);
    int chunk = prm->check_every > 0 ? prm->check_every : 25;
    double h[16], rr_prev = 0, it_prev = 0;
    // one iteration: 6 launches with fixed arguments (7 with the one-block total of a large
    // lattice), replayed as a graph
    auto iteration = [&]() -> int {
        int e;
        if ((e = clovinv64(ctx, 1, B.p, s.clov[1], B.T, 1.0, 1.0, cl, ctx->scal + S_DONE))) return e;
        if ((e = xpay64(ctx, 0, B.p, B.T, s.clov[0], mk2, B.t, 1.0, cl, B.part_a, ctx->scal + S_DONE))) return e;
        if (!inl && (e = launch_total<1>(ctx, B.part_a, nb, ctx->scal + S_PAP, ctx->scal + S_DONE))) return e;
        if ((e = clovinv64(ctx, 1, B.t, s.clov[1], B.T, -1.0, 1.0, cl, ctx->scal + S_DONE))) return e;
        // r -= alpha Khat p (the base x is not needed; it goes to scratch)
        launch_cg_hop4(ctx, cl, inl, nb, B.t, B.T, s.clov[0], mk2, B.p, B.Kx, B.r, B.part_b, B.part_a, rec, nshift);
        hipLaunchKernelGGL(k_ms_beta, dim3(1), dim3(kFinishThreads), 0, ctx->stream, B.part_b, nb, nshift, ctx->scal,
                           rec);
        hipLaunchKernelGGL(k_ms_update, dim3(nblocks(n, 256)), dim3(256), 0, ctx->stream, n, nshift, B.r, B.p, ptrs,
                           ptrs + nshift, rec, ctx->scal);
        LAUNCHCHK(ctx);
        return 0;
    };
    std::vector<uint64_t> key;
    key_add(key, 3);   // multi-shift iteration
    key_geom(key, g);
    key_add(key, nshift);
    for (const void *ptr : {(const void *)B.p, (const void *)B.T, (const void *)B.t, (const void *)B.r,
                            (const void *)B.Kx, (const void *)B.part_a, (const void *)B.part_b, (const void *)ptrs,
                            (const void *)ctx->U, (const void *)ctx->scal, (const void *)s.clov[0],
                            (const void *)s.clov[1]})
        key_add(key, ptr);
    key_add(key, mk2);
    key_add(key, (int)cl);
    for (;;) {
        if ((rc = graph_run(ctx, key, chunk, iteration))) return rc;
        if ((rc = read_state(ctx, h, 16))) return rc;
        if (h[S_DONE] != 0) break;
        if (prm->check_every <= 0) chunk = next_chunk(h[S_RR], h[S_THR], h[S_ITER], rr_prev, it_prev);
        rr_prev = h[S_RR];
        it_prev = h[S_ITER];
    }
    int iters = (int)h[S_ITER];
    double worst = 0;
    for (int k = 0; k < nshift; k++) {
        double res = 0;
        if ((rc = true_residual(ctx, op, b, (const double2 *)x_[k], make_double2(z[2 * k], z[2 * k + 1]), B, &res)))
            return rc;
        if (st && k < PFMP_MAX_SHIFTS) st->shift_res[k] = res;
        if (res > worst) worst = res;
    }
    auto t1 = std::chrono::steady_clock::now();
    if (st) {
        st->iters = iters;
        st->reliable_updates = 0;
        st->true_res = worst;
        st->seconds = std::chrono::duration<double>(t1 - t0).count();
        st->kmults = iters + nshift;
    }
    if (h[S_DONE] == 2) return set_err(ctx, PFMP_ERR_NOCONV, "cg_multishift: maxiter reached");
    return 0;
}
