// mixed.hip -- mixed-precision CG on Khat: FP32 inner iterations (FP32 links,
// clover and arithmetic; FP64 reductions and scalars) with FP64 reliable updates.
// Storage of the inner operator vectors (search direction p, Mhat p and the odd
// intermediates) is FP32 or FP16 with one FP32 scale per site; x and r stay FP32.
//
// The inner CG runs on (xs, rs, ps) in FP32.  When its residual has dropped by
// the factor delta since the last update, or reached the target, the device
// flags a reliable update: the host adds xs into the FP64 solution, recomputes the
// FP64 true residual r = b - Khat x, restarts rs from it and keeps the search
// direction ps.  The solve ends only when the FP64 true residual meets tol.
#include <chrono>
#include <cmath>
#include <type_traits>

#include "hop.h"

namespace {

enum { M_RR = 0, M_THR, M_DTHR, M_PAP, M_ALPHA, M_BETA, M_ITER, M_DONE, M_MAXIT, M_RROLD, M_ITNEXT };
constexpr int kMixBase = 4096;    // device scalar slots of this solver (ctx->scal + kMixBase)

__device__ __forceinline__ double block_total_m(const double *__restrict__ partials, int nparts)
{
    __shared__ double sh[kRedBlock / 64];
    double s = 0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) s += partials[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0;
    for (int k = 0; k < kRedBlock / 64; k++) t += sh[k];
    return t;
}

// (re)start: rr = |r|^2 of the FP64 residual (partials), thresholds
__global__ __launch_bounds__(kRedBlock) void k_m_restart(const double *__restrict__ partials, int nparts,
                                                         double tol2bb, double delta2, int maxiter, int first,
                                                         double *__restrict__ st)
{
    double rr = block_total_m(partials, nparts);
    if (threadIdx.x == 0) {
        // the iteration that flagged the update skipped p = r + beta p; redo it with
        // the true residual: beta' = |r_true|^2 / |r_prev|^2, |r_prev|^2 = rr_inner / beta
        if (!first) st[M_BETA] = rr * st[M_BETA] / st[M_RR];
        st[M_RR] = rr;
        st[M_THR] = tol2bb;
        st[M_DTHR] = delta2 * rr;
        if (first) st[M_ITER] = 0;
        st[M_MAXIT] = maxiter;
        st[M_DONE] = 0;
    }
}

// FP32 Khat p from t = Mhat p and T' (as in the FP64 solver), fused with
// x += alpha p, r -= alpha Khat p and the FP64 |r+|^2 partials.  alpha = |r|^2 / <p, Khat p>
// with <p, Khat p> formed from the stage-2 partials by every block (INL) or read from M_PAP
// (totalled by a one-block kernel); block 0 records alpha and, with INL, <p, Khat p>, |r|^2
// (M_RROLD) and the next iteration count (M_ITNEXT) for the p update.
template <int CLOV, int LM, int INL, typename S, typename UL, typename CL>
__global__ __launch_bounds__(kBlock) void k_m_hop4(Geom g, const S t, const S T, UL U, CL cl, float a, const S p,
                                                   float2 *__restrict__ x, float2 *__restrict__ r,
                                                   double *__restrict__ st, double *__restrict__ partials,
                                                   const double *__restrict__ part_pap, int npap)
{
    if (st[M_DONE] != 0) return;
    double pap;
    if (INL) {
        double tp[1];
        partials_total<kBlock, 1, kInlineChunks>(part_pap, npap, tp);
        pap = tp[0];
    } else {
        pap = st[M_PAP];
    }
    const double alpha_d = st[M_RR] / pap;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st[M_ALPHA] = alpha_d;
        if (INL) {
            st[M_PAP] = pap;
            st[M_RROLD] = st[M_RR];
            st[M_ITNEXT] = st[M_ITER] + 1;
        }
    }
    const int tt = xcd_site(2 * g.Vh);
    double nrm = 0;
    if (tt >= 0) {
        const int i = tile_site(g, tt >> 1), hb = tt & 1;
        float2 acc[6], tv[6], at[6], pp[6];
        hop_pair<LM, float2>(g, 0, i, hb, T, U, 1.f, acc);
        // site-local vectors: non-temporal when the links stream (large lattices; FP16
        // records stay cached)
        constexpr int ST = (LM >> 1) & 1;
        load_block_st<ST>(t, g.Vh, i, hb, -1.f, tv);
        load_block_st<ST>(p, g.Vh, i, hb, 1.f, pp);
        if (CLOV) clover_block<float, float2>(cl, g.Vh, i, hb, tv, at);
        const float alpha = (float)alpha_d;
        const long Vh = g.Vh;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            float2 base = CLOV ? at[k] : tv[k];
            float2 kp = make_float2(fmadd(a, acc[k].x, base.x), fmadd(a, acc[k].y, base.y));
            if (hb) kp = cneg(kp);
            const long e = (long)(6 * hb + k) * Vh + i;
            float2 pv = pp[k], xv = ld_st<ST>(x + e), rv = ld_st<ST>(r + e);
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

// The stop decision from |r+|^2 (1: inner residual at the target, 3: dropped by delta ->
// reliable update, 2: iteration limit) and beta = |r+|^2 / |r|^2
__device__ __forceinline__ int m_decide(double rr, double it, const double *st)
{
    return rr <= st[M_THR] ? 1 : (rr <= st[M_DTHR] ? 3 : (it >= st[M_MAXIT] ? 2 : 0));
}

// |r+|^2 from the stage-4 partials, the decision and beta; one workgroup (many partials)
__global__ __launch_bounds__(kFinishThreads) void k_m_finish_rr(const double *__restrict__ part, int n,
                                                               double *__restrict__ st)
{
    if (st[M_DONE] != 0) return;
    double t[1];
    partials_total<kFinishThreads, 1, kMaxChunks>(part, n, t);
    if (threadIdx.x == 0) {
        const double rr = t[0], it = st[M_ITER] + 1;
        st[M_BETA] = rr / st[M_RR];
        st[M_RR] = rr;
        st[M_ITER] = it;
        st[M_DONE] = m_decide(rr, it, st);
    }
}

// p = r + beta p, two lanes per site (lane hb: chiral block hb; FP16 storage takes the site's
// scale over both lanes' blocks, so the stored values are those of a one-lane update).  With
// part_rr (INL): every block forms |r+|^2 from the stage-4 partials and takes the stop
// decision from it and the iteration count M_ITNEXT (written by stage 4), the same in every
// block, and skips the update on a stop, which the restart after a reliable update relies
// on; block 0 records the state.  Without part_rr: beta and the decision from st (one-block
// total, or the restart).  st == nullptr: p = r.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_m_update_p(Geom g, const float2 *__restrict__ r, S p,
                                                       double *__restrict__ st, const double *__restrict__ part_rr,
                                                       int nrr)
{
    if (st && st[M_DONE] != 0) return;
    double bd = st ? st[M_BETA] : 0.0;
    if (part_rr) {
        double tr[1];
        partials_total<kBlock, 1, kInlineChunks>(part_rr, nrr, tr);
        const double rr = tr[0], it = st[M_ITNEXT];
        const int done = m_decide(rr, it, st);
        bd = rr / st[M_RROLD];
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st[M_BETA] = bd;
            st[M_RR] = rr;
            st[M_ITER] = it;
            st[M_DONE] = done;
        }
        if (done) return;
    }
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t >> 1, hb = t & 1;
    if (i >= g.Vh) return;   // both lanes of a pair leave together
    float2 rv[6], pv[6];
    load_block(r, g.Vh, i, hb, 1.f, rv);
    if (st) {
        const float b = (float)bd;
        load_block(p, g.Vh, i, hb, 1.f, pv);
#pragma unroll
        for (int k = 0; k < 6; k++) rv[k] = make_float2(fmadd(b, pv[k].x, rv[k].x), fmadd(b, pv[k].y, rv[k].y));
    }
    store_block(p, g.Vh, i, hb, 1.f, rv);
}

// x += xs (FP64 += FP32), xs = 0
__global__ void k_m_accum(long n, float2 *__restrict__ xs, double2 *__restrict__ x)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    float2 v = xs[t];
    double2 w = x[t];
    x[t] = make_double2(w.x + (double)v.x, w.y + (double)v.y);
    xs[t] = make_float2(0.f, 0.f);
}

// r = b - Kx (FP64); rs = (float) r; |r|^2 partials (grid-stride)
__global__ __launch_bounds__(kRedBlock) void k_m_residual(long n, const double2 *__restrict__ b,
                                                          const double2 *__restrict__ Kx, float2 *__restrict__ rs,
                                                          double *__restrict__ partials)
{
    double s = 0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        double2 r = csub(b[t], Kx[t]);
        s += r.x * r.x + r.y * r.y;
        rs[t] = make_float2((float)r.x, (float)r.y);
    }
    __shared__ double sh[kRedBlock / 64];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0;
        for (int k = 0; k < kRedBlock / 64; k++) v += sh[k];
        partials[blockIdx.x] = v;
    }
}

}  // namespace

// Inner-solver storage: FP32 spinors with the FP32 links and clover, or FP16 spinors
// (per-site scale) with the FP16 links and clover; arithmetic in FP32 either way.
template <typename S, bool HL = true> struct Store;
template <> struct Store<float2 *, true> {
    using In = const float2 *;
    using UL = const float2 *;
    using CL = const float *;
    static size_t bytes(long Vh) { return 8L * 12 * Vh; }
    static float2 *make(void *p, long) { return (float2 *)p; }
    static UL links(const pfmp_ctx *ctx) { return ctx->Uf; }
    static CL clover(const OpSlot &s, int p) { return s.clovf[p]; }
};
// FP16 spinor storage with the FP16 copies of the links and clover (HL) or the FP32 ones
template <> struct Store<HalfField, true> {
    using In = HalfField;
    using UL = HalfLinks;
    using CL = HalfClover;
    static size_t bytes(long Vh) { return 4L * 12 * Vh + 4L * Vh; }
    static HalfField make(void *p, long Vh) { return HalfField{(H3 *)p, (float *)((char *)p + 4L * 12 * Vh)}; }
    static UL links(const pfmp_ctx *ctx) { return HalfLinks{(const __half2 *)ctx->Uh}; }
    static CL clover(const OpSlot &s, int p) { return HalfClover{(const H3 *)s.clovh[p]}; }
};
template <> struct Store<HalfField, false> {
    using In = HalfField;
    using UL = const float2 *;
    using CL = const float *;
    static size_t bytes(long Vh) { return Store<HalfField, true>::bytes(Vh); }
    static HalfField make(void *p, long Vh) { return Store<HalfField, true>::make(p, Vh); }
    static UL links(const pfmp_ctx *ctx) { return ctx->Uf; }
    static CL clover(const OpSlot &s, int p) { return s.clovf[p]; }
};

template <typename S, bool HL = true>
static int mixed_impl(pfmp_ctx *ctx, int op, const void *b_, void *x_, const pfmp_solver_params *prm,
                      pfmp_solver_stats *st)
{
    using St = Store<S, HL>;
    using In = typename St::In;
    using UL = typename St::UL;
    using CL = typename St::CL;
    auto t0 = std::chrono::steady_clock::now();
    const Geom &g = ctx->g;
    OpSlot &s = ctx->ops[op];
    const UL links = St::links(ctx);
    const CL clo0 = St::clover(s, 0), clo1 = St::clover(s, 1);
    const long n = 12L * g.Vh;
    const size_t vb = sizeof(double) * spinor_reals(g), fb = vb / 2;
    const int nb = op_nparts(g);
    double2 *Kx = (double2 *)ws_alloc(ctx, vb, 8), *te = (double2 *)ws_alloc(ctx, vb, 6),
            *to = (double2 *)ws_alloc(ctx, vb, 7);
    const size_t sb = St::bytes(g.Vh);
    float2 *rs = (float2 *)ws_alloc(ctx, fb, 27), *xs = (float2 *)ws_alloc(ctx, fb, 29);
    void *pb = ws_alloc(ctx, sb, 28), *tb = ws_alloc(ctx, sb, 30), *Tb = ws_alloc(ctx, sb, 31);
    double *part_a = (double *)ws_alloc(ctx, sizeof(double) * (nb + 64), 9);
    double *part_b = (double *)ws_alloc(ctx, sizeof(double) * (nb + 64), 10);
    if (!Kx || !te || !to || !rs || !xs || !pb || !tb || !Tb || !part_a || !part_b)
        return set_err(ctx, PFMP_ERR_OOM, "mixed solver workspace");
    S ps = St::make(pb, g.Vh), ts = St::make(tb, g.Vh), Ts = St::make(Tb, g.Vh);
    const double2 *b = (const double2 *)b_;
    double2 *x = (double2 *)x_;
    double *sc = ctx->scal + kMixBase;
    // default trigger: FP32 storage keeps the recurrence close to the true residual, so rare updates
    // (a 100x drop) cost nothing in iterations; FP16 storage drifts sooner and wants one per 10x drop
    const double delta = prm->delta > 0 ? prm->delta : (std::is_same<S, float2 *>::value ? 0.01 : 0.1);
    const bool cl = s.csw != 0;
    const float mk2 = (float)(-s.kappa * s.kappa);
    const bool inl = totals_inline(nb);
    int rc;
    HIPCHK(ctx, hipMemsetAsync(x, 0, vb, ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(xs, 0, fb, ctx->stream));
    HIPCHK(ctx, hipMemsetAsync(Kx, 0, vb, ctx->stream));
    double bb;
    if ((rc = launch_norm2(ctx, b, n, ctx->red))) return rc;
    if ((rc = red_finish(ctx, ctx->red, ctx->nblk_red, 1, &bb))) return rc;
    const double tol2bb = prm->tol * prm->tol * bb;
    if (bb == 0) {   // b = 0: x = 0 solves it exactly (and alpha would be 0 / 0)
        if (st) *st = pfmp_solver_stats{};
        return 0;
    }
    // r = b, rs = (float) b, p = rs
    hipLaunchKernelGGL(k_m_residual, dim3(ctx->nblk_red), dim3(kRedBlock), 0, ctx->stream, n, b, Kx, rs, ctx->red);
    hipLaunchKernelGGL((k_m_update_p<S>), dim3(nblocks(2L * g.Vh, kBlock)), dim3(kBlock), 0, ctx->stream, g, rs, ps,
                       (double *)nullptr, (const double *)nullptr, 0);
    hipLaunchKernelGGL(k_m_restart, dim3(1), dim3(kRedBlock), 0, ctx->stream, ctx->red, ctx->nblk_red, tol2bb,
                       delta * delta, prm->maxiter, 1, sc);
    LAUNCHCHK(ctx);
    int chunk = prm->check_every > 0 ? prm->check_every : 16;
    int updates = 0, kmults = 0, last_iter = 0;
    double h[16], res = 0;
    // one inner iteration: 5 launches with fixed arguments, replayed as a graph
    auto iteration = [&]() -> int {
        int e;
        if ((e = launch_clovinv<float2, float, In, S, UL, CL>(ctx, 1, ps, links, clo1, Ts, 1.f, 1.f, cl, sc + M_DONE)))
            return e;
        if ((e = launch_xpay<float2, float, In, In, S, UL, CL>(ctx, 0, ps, Ts, links, clo0, mk2, ts, 1.f, cl, part_a,
                                                                sc + M_DONE)))
            return e;
        if (!inl && (e = launch_total<1>(ctx, part_a, nb, sc + M_PAP, sc + M_DONE))) return e;
        if ((e = launch_clovinv<float2, float, In, S, UL, CL>(ctx, 1, ts, links, clo1, Ts, -1.f, 1.f, cl,
                                                               sc + M_DONE)))
            return e;
#define MHOP4(CV, LM, IN)                                                                                       \
    hipLaunchKernelGGL((k_m_hop4<CV, LM, IN, In, UL, CL>), dim3(nb), dim3(kBlock), 0, ctx->stream, g, ts, Ts, links, \
                       clo0, mk2, ps, xs, rs, sc, part_b, part_a, nb)
#define MHOP4_1(LM) if (inl) MHOP4(1, LM, 1); else MHOP4(1, LM, 0)
#define MHOP4_0(LM) if (inl) MHOP4(0, LM, 1); else MHOP4(0, LM, 0)
        if (cl) { PFMP_LM_SWITCH(link_mode(g), MHOP4_1) }
        else { PFMP_LM_SWITCH(link_mode(g), MHOP4_0) }
#undef MHOP4_1
#undef MHOP4_0
#undef MHOP4
        if (!inl)
            hipLaunchKernelGGL(k_m_finish_rr, dim3(1), dim3(kFinishThreads), 0, ctx->stream, part_b, nb, sc);
        hipLaunchKernelGGL((k_m_update_p<S>), dim3(nblocks(2L * g.Vh, kBlock)), dim3(kBlock), 0, ctx->stream, g, rs, ps,
                           sc, inl ? (const double *)part_b : (const double *)nullptr, nb);
        LAUNCHCHK(ctx);
        return 0;
    };
    std::vector<uint64_t> key;
    key_add(key, 2 + (int)sizeof(S));   // mixed-precision iteration, storage type
    key_add(key, (int)HL);
    key_geom(key, g);
    for (const void *ptr : {(const void *)pb, (const void *)tb, (const void *)Tb, (const void *)xs, (const void *)rs, (const void *)part_a,
                            (const void *)part_b, (const void *)sc, (const void *)ctx->Uf, (const void *)ctx->Uh,
                            (const void *)s.clovf[0], (const void *)s.clovf[1], (const void *)s.clovh[0],
                            (const void *)s.clovh[1]})
        key_add(key, ptr);
    key_add(key, mk2);
    key_add(key, (int)cl);
    for (;;) {
        if ((rc = graph_run(ctx, key, chunk, iteration))) return rc;
        HIPCHK(ctx, hipMemcpyAsync(ctx->red_host, sc, sizeof(double) * 16, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        for (int k = 0; k < 16; k++) h[k] = ctx->red_host[k];
        if (h[M_DONE] == 0) {
            if (prm->check_every <= 0) chunk = 4;   // close in on the flagged iteration
            continue;
        }
        // reliable update in FP64
        hipLaunchKernelGGL(k_m_accum, dim3(nblocks(n, 256)), dim3(256), 0, ctx->stream, n, xs, x);
        if ((rc = op_apply_K(ctx, op, x, Kx, te, to, nullptr))) return rc;
        kmults++;
        updates++;
        hipLaunchKernelGGL(k_m_residual, dim3(ctx->nblk_red), dim3(kRedBlock), 0, ctx->stream, n, b, Kx, rs,
                           ctx->red);
        double rr;
        if ((rc = red_finish(ctx, ctx->red, ctx->nblk_red, 1, &rr))) return rc;
        res = bb > 0 ? std::sqrt(rr / bb) : 0;
        if (rr <= tol2bb || h[M_DONE] == 2) break;
        hipLaunchKernelGGL(k_m_restart, dim3(1), dim3(kRedBlock), 0, ctx->stream, ctx->red, ctx->nblk_red, tol2bb,
                           delta * delta, prm->maxiter, 0, sc);
        hipLaunchKernelGGL((k_m_update_p<S>), dim3(nblocks(2L * g.Vh, kBlock)), dim3(kBlock), 0, ctx->stream, g, rs, ps,
                           sc, (const double *)nullptr, 0);
        LAUNCHCHK(ctx);
        // the next chunk: about as long as the last stretch between reliable updates
        if (prm->check_every <= 0) {
            const int stretch = (int)h[M_ITER] - last_iter;
            chunk = stretch > 4 ? stretch - 1 : 4;
        }
        last_iter = (int)h[M_ITER];
    }
    auto t1 = std::chrono::steady_clock::now();
    if (st) {
        st->iters = (int)h[M_ITER];
        st->reliable_updates = updates;
        st->true_res = res;
        st->seconds = std::chrono::duration<double>(t1 - t0).count();
        st->kmults = (long long)h[M_ITER] + kmults;
    }
    if (!(res <= prm->tol)) return set_err(ctx, PFMP_ERR_NOCONV, "cg_solve (mixed): maxiter reached");
    return 0;
}

int cg_solve_mixed(pfmp_ctx *ctx, int op, const void *b, void *x, const pfmp_solver_params *p, pfmp_solver_stats *st)
{
    if (p->prec == PFMP_F32) return mixed_impl<float2 *>(ctx, op, b, x, p, st);
    if (p->prec == PFMP_F16)
        return ctx->half_links ? mixed_impl<HalfField, true>(ctx, op, b, x, p, st)
                               : mixed_impl<HalfField, false>(ctx, op, b, x, p, st);
    return set_err(ctx, PFMP_ERR_ARG, "cg_solve: unsupported precision");
}
