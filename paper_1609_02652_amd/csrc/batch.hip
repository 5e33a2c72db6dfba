// batch.hip -- multi-RHS operator and CG: k right-hand sides, each with its own
// operator slot (kappa, clover), in one launch per stage.
//
// Each workgroup serves one right-hand side (so every pointer and scalar of the rhs is
// uniform in the workgroup) with the two-lanes-per-site kernels of the single-RHS
// operator.  The n workgroups that cover the same block of sites for the n right-hand
// sides are consecutive in the XCD-aware block order, so they run together on one XCD
// and every link is fetched once into its L2 for all n.  Per-rhs CG scalars and
// convergence flags live on the device; a converged rhs stops touching memory.
// Reductions: one FP64 partial per workgroup and rhs, indexed by its site block, totalled
// per rhs by one-workgroup kernels in the fixed order of the single-RHS solver
// (partials_total), so an FP64 batched solve gives each right-hand side the bits of its
// single-RHS solve.
//
// The kernels are written once for FP64 and FP32 fields.  The FP64 batched CG is plain
// CG on every right-hand side; the mixed-precision one is defect correction: FP64
// residuals r_r = b_r - Khat x_r, the batched FP32 CG (FP32 links and clover) on
// r_r / |r_r| to a relative 2e-6 or what the remaining reduction needs, x_r += |r_r| e_r
// in FP64, until every FP64 residual is at the tolerance.
#include <chrono>
#include <cmath>

#include "hop.h"

namespace {

constexpr int kMaxRhs = 8;
enum { B_RR = 0, B_THR, B_PAP, B_ALPHA, B_BETA, B_ITER, B_DONE, B_MAXIT, B_NSLOT = 8 };
constexpr int kBatchBase = 5120;   // per-rhs scalar records at ctx->scal + kBatchBase + 8 r

template <typename R>
struct BatchT {
    int k;                          // stride of the partials (= n)
    int n;                          // right-hand sides
    int nsb;                        // site blocks (two lanes per site, kBlock lanes per block)
    int pstride;                    // partials per right-hand side (>= nsb)
    const R *clo[kMaxRhs];          // A_oo^-1 of each rhs's operator
    const R *cle[kMaxRhs];          // A_ee
    R a[kMaxRhs];                   // -kappa^2
    int clov[kMaxRhs];
};

template <typename C>
struct VecsT {
    const C *in[kMaxRhs];
    C *out[kMaxRhs];
};

// Workgroup of this launch: logical workgroup lb = site block * n + rhs (XCD-aware
// order).  False for the padding workgroups past the end (a whole workgroup).
template <typename R>
__device__ __forceinline__ bool wg_item(const BatchT<R> &b, int *sb, int *r)
{
    const int lb = xcd_block();
    if (lb >= b.nsb * b.n) return false;
    *r = lb % b.n;
    *sb = lb / b.n;
    return true;
}

// out_r = [g5] A_oo^-1 D_oe [g5] in_r
template <typename C, typename R, int CLOV, int LM>
__global__ __launch_bounds__(kBlock) void k_b_clovinv(Geom g, BatchT<R> b, VecsT<C> v, const C *__restrict__ U,
                                                      R gin, R gout, const double *__restrict__ st)
{
    int sb, r;
    if (!wg_item(b, &sb, &r)) return;
    if (st && st[8 * r + B_DONE] != 0) return;
    const int t = sb * kBlock + threadIdx.x;
    if (t >= 2 * g.Vh) return;
    const int i = tile_site(g, t >> 1), hb = t & 1;
    C blk[6];
    hop_pair<LM, C>(g, 1, i, hb, v.in[r], U, gin, blk);
    if (CLOV) {
        C tq[6];
        clover_block<R, C>(b.clo[r], g.Vh, i, hb, blk, tq);
        store_block(v.out[r], g.Vh, i, hb, gout, tq);
    } else {
        store_block(v.out[r], g.Vh, i, hb, gout, blk);
    }
}

// out_r = [g5] (A_ee [g5] x_r + a_r D_eo t_r) in the single-RHS stage's arithmetic; with
// partials, the |out_r|^2 partials of each rhs, indexed by site block
template <typename C, typename R, int CLOV, int LM>
__global__ __launch_bounds__(kBlock) void k_b_xpay(Geom g, BatchT<R> b, VecsT<C> x, VecsT<C> t,
                                                   const C *__restrict__ U, R gs, const double *__restrict__ st,
                                                   double *__restrict__ partials)
{
    int sb, r;
    if (!wg_item(b, &sb, &r)) return;
    if (st && st[8 * r + B_DONE] != 0) return;
    const int tt = sb * kBlock + threadIdx.x;
    double nrm = 0;
    if (tt < 2 * g.Vh) {
        const int i = tile_site(g, tt >> 1), hb = tt & 1;
        C acc[6], xv[6], ax[6];
        hop_pair<LM, C>(g, 0, i, hb, t.in[r], U, (R)1, acc);
        load_block(x.in[r], g.Vh, i, hb, gs, xv);
        if (CLOV) clover_block<R, C>(b.cle[r], g.Vh, i, hb, xv, ax);
        const R a = b.a[r];
#pragma unroll
        for (int k = 0; k < 6; k++) {
            C base = CLOV ? ax[k] : xv[k];
            acc[k] = mk<C>(fmadd(a, acc[k].x, base.x), fmadd(a, acc[k].y, base.y));
            cnorm_acc(nrm, acc[k]);
        }
        store_block(x.out[r], g.Vh, i, hb, gs, acc);
    }
    if (partials) {
        const double v[1] = {nrm};
        partials_store_at<kBlock, 1>(v, partials + (long)r * b.pstride, sb);
    }
}

// CG stage 4 in the single-RHS arithmetic: Kp_r from t_r and T'_r; x_r += alpha_r p_r;
// r_r -= alpha_r Kp_r; the |r_r|^2 partials of each rhs, indexed by site block
template <typename C, typename R, int CLOV, int LM>
__global__ __launch_bounds__(kBlock) void k_b_hop4(Geom g, BatchT<R> b, VecsT<C> t, VecsT<C> T, VecsT<C> p,
                                                   VecsT<C> x, VecsT<C> rr, const C *__restrict__ U,
                                                   const double *__restrict__ st, double *__restrict__ partials)
{
    int sb, r;
    if (!wg_item(b, &sb, &r)) return;
    const double *s = st + 8 * r;
    if (s[B_DONE] != 0) return;
    const double alpha_d = s[B_RR] / s[B_PAP];
    const int tt = sb * kBlock + threadIdx.x;
    double nrm = 0;
    if (tt < 2 * g.Vh) {
        const int i = tile_site(g, tt >> 1), hb = tt & 1;
        C acc[6], tv[6], at[6];
        hop_pair<LM, C>(g, 0, i, hb, T.in[r], U, (R)1, acc);
        load_block(t.in[r], g.Vh, i, hb, (R)-1, tv);
        if (CLOV) clover_block<R, C>(b.cle[r], g.Vh, i, hb, tv, at);
        const R alpha = (R)alpha_d, a = b.a[r];
        const long Vh = g.Vh;
        const C *pp = p.in[r];
        C *xx = x.out[r], *rv_ = rr.out[r];
#pragma unroll
        for (int k = 0; k < 6; k++) {
            C base = CLOV ? at[k] : tv[k];
            C kp = mk<C>(fmadd(a, acc[k].x, base.x), fmadd(a, acc[k].y, base.y));
            if (hb) kp = cneg(kp);
            const long e = (long)(6 * hb + k) * Vh + i;
            C pv = pp[e], xv = xx[e], rv = rv_[e];
            xv.x = fmadd(alpha, pv.x, xv.x); xv.y = fmadd(alpha, pv.y, xv.y);
            rv.x = fmadd(-alpha, kp.x, rv.x); rv.y = fmadd(-alpha, kp.y, rv.y);
            xx[e] = xv;
            rv_[e] = rv;
            cnorm_acc(nrm, rv);
        }
    }
    const double v[1] = {nrm};
    partials_store_at<kBlock, 1>(v, partials + (long)r * b.pstride, sb);
}

// <p, Khat p> of each running rhs from its partials (the single-RHS solver's order)
__global__ __launch_bounds__(kFinishThreads) void k_b_pap(const double *__restrict__ partials, int nparts,
                                                         int pstride, int n, double *__restrict__ st)
{
    for (int r = 0; r < n; r++) {
        if (st[8 * r + B_DONE] != 0) continue;
        double t[1];
        partials_total<kFinishThreads, 1, kMaxChunks>(partials + (long)r * pstride, nparts, t);
        if (threadIdx.x == 0) st[8 * r + B_PAP] = t[0];
    }
}

// |r+|^2, beta and the stop decision of each running rhs (the single-RHS solver's order)
__global__ __launch_bounds__(kFinishThreads) void k_b_beta(const double *__restrict__ partials, int nparts,
                                                          int pstride, int n, double *__restrict__ st)
{
    for (int r = 0; r < n; r++) {
        double *s = st + 8 * r;
        if (s[B_DONE] != 0) continue;
        double t[1];
        partials_total<kFinishThreads, 1, kMaxChunks>(partials + (long)r * pstride, nparts, t);
        if (threadIdx.x == 0) {
            const double rr = t[0], it = s[B_ITER] + 1;
            s[B_BETA] = rr / s[B_RR];
            s[B_RR] = rr;
            s[B_ITER] = it;
            s[B_DONE] = rr <= s[B_THR] ? 1 : (it >= s[B_MAXIT] ? 2 : 0);
        }
        __syncthreads();
    }
}

// p_r = r_r + beta_r p_r for the right-hand sides still running
template <typename C>
__global__ void k_b_update_p(Geom g, int nrhs, VecsT<C> rr, VecsT<C> p, const double *__restrict__ st)
{
    using R = decltype(C::x);
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    long n = 12L * g.Vh;
    int r = (int)(t / n);
    long e = t - (long)r * n;
    if (r >= nrhs || st[8 * r + B_DONE] != 0) return;
    const R beta = (R)st[8 * r + B_BETA];
    C rv = rr.in[r][e], pv = p.out[r][e];
    p.out[r][e] = mk<C>(fmadd(beta, pv.x, rv.x), fmadd(beta, pv.y, rv.y));
}

// ---------------------------------------------------------------- one workgroup, NR rhs
//
// The same stages with the NR right-hand sides of a launch (rhs r0 .. r0 + NR - 1) in one
// lane pair per site: each leg's link is loaded once and applied to the NR neighbour half
// spinors, with the single-RHS leg arithmetic (leg_apply) for each, so every rhs gets the
// bits of its single-RHS stage.  A converged rhs is skipped by the whole workgroup.

// active right-hand sides of the launch (uniform in the workgroup)
template <int NR>
__device__ __forceinline__ void rhs_active(const double *__restrict__ st, int r0, bool *act)
{
#pragma unroll
    for (int q = 0; q < NR; q++) act[q] = !st || st[8 * (r0 + q) + B_DONE] == 0;
}

// Memory hints of the multi-rhs kernels: when the context streams links (large lattices), their
// outputs, the spinors read only at the site itself and the FP64 links, all touched once per
// launch, go through non-temporal loads and stores, leaving L2 to the neighbour spinors, which
// four right-hand sides make four times as large (32^3 x 64, 4 rhs of one operator: K-hat per
// rhs 1 102 -> 1 013 us in FP64, 592 -> 578 us in FP32, the same bits).

// the clover blocks of a launch's rhs: fetched once when every rhs of the launch uses the same
// field (one operator), else per rhs (uniform in the workgroup)
template <int NR, typename R>
__device__ __forceinline__ bool clover_shared(const R *const *cl, int r0)
{
    bool same = true;
#pragma unroll
    for (int q = 1; q < NR; q++) same = same && cl[r0 + q] == cl[r0];
    return same;
}

template <int MU, int DIR, int LM, int NR, typename C, typename UL>
__device__ __forceinline__ void legs_multi(const Geom &g, int pout, int i, const int *c, int hb,
                                           const C *const *in, UL U, decltype(C::x) gs, const bool *act,
                                           C (*up)[3], C (*loA)[3], C (*loB)[3])
{
    int s;
    const int j = eo_neighbour(g, c, MU, DIR ? -1 : +1, &s);
    const int qs = MU < 2 ? 3 - hb : 2 + hb;
    const int lp = DIR ? 1 - pout : pout;
    Leg<C, const C *, UL, LM> l[NR];
    l[0].lk.template load<(LM >> 1) & 1>(lshift(U, ((long)(lp * 4 + MU) * 9) * g.Vh), g.Vh, DIR ? j : i);
#pragma unroll
    for (int q = 0; q < NR; q++) {
        if (q > 0) l[q].lk = l[0].lk;
        l[q].sg = (decltype(C::x))s;
        if (act[q]) l[q].sp.load(in[q], g.Vh, j, 3 * hb, 3 * qs);
    }
#pragma unroll
    for (int q = 0; q < NR; q++)
        if (act[q]) leg_apply<MU, DIR, LM, C>(l[q], hb, gs, up[q], loA[q], loB[q]);
}

// D_hop in_q for the NR rhs (block hb of the result at output site i), as hop_pair
template <int LM, int NR, typename C, typename UL>
__device__ __forceinline__ void hop_multi(const Geom &g, int pout, int i, int hb, const C *const *in, UL U,
                                          decltype(C::x) gs, const bool *act, C (*blk)[6])
{
    int c[4];
    eo_coords(g, pout, i, c);
    C up[NR][3], loA[NR][3], loB[NR][3];
#pragma unroll
    for (int q = 0; q < NR; q++)
#pragma unroll
        for (int a = 0; a < 3; a++) up[q][a] = loA[q][a] = loB[q][a] = mk<C>(0, 0);
    legs_multi<0, 0, LM, NR>(g, pout, i, c, hb, in, U, gs, act, up, loA, loB);
    legs_multi<0, 1, LM, NR>(g, pout, i, c, hb, in, U, gs, act, up, loA, loB);
    legs_multi<1, 0, LM, NR>(g, pout, i, c, hb, in, U, gs, act, up, loA, loB);
    legs_multi<1, 1, LM, NR>(g, pout, i, c, hb, in, U, gs, act, up, loA, loB);
    legs_multi<2, 0, LM, NR>(g, pout, i, c, hb, in, U, gs, act, up, loA, loB);
    legs_multi<2, 1, LM, NR>(g, pout, i, c, hb, in, U, gs, act, up, loA, loB);
    legs_multi<3, 0, LM, NR>(g, pout, i, c, hb, in, U, gs, act, up, loA, loB);
    legs_multi<3, 1, LM, NR>(g, pout, i, c, hb, in, U, gs, act, up, loA, loB);
#pragma unroll
    for (int q = 0; q < NR; q++) {
        C x[6];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            x[a] = hb ? up[q][a] : loB[q][a];
            x[3 + a] = hb ? up[q][a] : loA[q][a];
        }
#pragma unroll
        for (int k = 0; k < 6; k++) x[k] = mk<C>(pair_swap(x[k].x), pair_swap(x[k].y));
#pragma unroll
        for (int a = 0; a < 3; a++) {
            blk[q][a] = hb ? cadd(loA[q][a], x[a]) : up[q][a];
            blk[q][3 + a] = hb ? cadd(loB[q][a], x[3 + a]) : x[a];
        }
    }
}

// out_r = [g5] A_oo^-1 D_oe [g5] in_r for r = r0 .. r0 + NR - 1
template <typename C, typename R, int CLOV, int LM, int NR>
__global__ __launch_bounds__(kBlock) void k_bm_clovinv(Geom g, BatchT<R> b, VecsT<C> v, const C *__restrict__ U,
                                                       R gin, R gout, const double *__restrict__ st, int r0)
{
    const int tt = xcd_site(2 * g.Vh);
    if (tt < 0) return;
    bool act[NR];
    rhs_active<NR>(st, r0, act);
    const int i = tile_site(g, tt >> 1), hb = tt & 1;
    C blk[NR][6];
    hop_multi<LM, NR>(g, 1, i, hb, v.in + r0, U, gin, act, blk);
    const bool same = clover_shared<NR>(b.clo, r0);
    R d[6];
    C o[15];
    if (CLOV && same) clover_fetch(b.clo[r0], g.Vh, i, hb, d, o);
#pragma unroll
    for (int q = 0; q < NR; q++) {
        if (!act[q]) continue;
        if (CLOV) {
            C tq[6];
            if (!same) clover_fetch(b.clo[r0 + q], g.Vh, i, hb, d, o);
            clover_mul(d, o, blk[q], tq);
            store_block_st<(LM >> 1) & 1>(v.out[r0 + q], g.Vh, i, hb, gout, tq);
        } else {
            store_block_st<(LM >> 1) & 1>(v.out[r0 + q], g.Vh, i, hb, gout, blk[q]);
        }
    }
}

// out_r = [g5] (A_ee [g5] x_r + a_r D_eo t_r); with partials, the |out_r|^2 partials
template <typename C, typename R, int CLOV, int LM, int NR>
__global__ __launch_bounds__(kBlock) void k_bm_xpay(Geom g, BatchT<R> b, VecsT<C> x, VecsT<C> t,
                                                    const C *__restrict__ U, R gs, const double *__restrict__ st,
                                                    double *__restrict__ partials, int r0)
{
    const int tt = xcd_site(2 * g.Vh);
    bool act[NR];
    rhs_active<NR>(st, r0, act);
    double nrm[NR];
#pragma unroll
    for (int q = 0; q < NR; q++) nrm[q] = 0;
    if (tt >= 0) {
        const int i = tile_site(g, tt >> 1), hb = tt & 1;
        C acc[NR][6];
        hop_multi<LM, NR>(g, 0, i, hb, t.in + r0, U, (R)1, act, acc);
        const bool same = clover_shared<NR>(b.cle, r0);
        R d[6];
        C o[15];
        if (CLOV && same) clover_fetch(b.cle[r0], g.Vh, i, hb, d, o);
#pragma unroll
        for (int q = 0; q < NR; q++) {
            if (!act[q]) continue;
            C xv[6], ax[6];
            load_block_st<(LM >> 1) & 1>(x.in[r0 + q], g.Vh, i, hb, gs, xv);
            if (CLOV) {
                if (!same) clover_fetch(b.cle[r0 + q], g.Vh, i, hb, d, o);
                clover_mul(d, o, xv, ax);
            }
            const R a = b.a[r0 + q];
#pragma unroll
            for (int k = 0; k < 6; k++) {
                C base = CLOV ? ax[k] : xv[k];
                acc[q][k] = mk<C>(fmadd(a, acc[q][k].x, base.x), fmadd(a, acc[q][k].y, base.y));
                cnorm_acc(nrm[q], acc[q][k]);
            }
            store_block_st<(LM >> 1) & 1>(x.out[r0 + q], g.Vh, i, hb, gs, acc[q]);
        }
    }
    if (partials)
#pragma unroll
        for (int q = 0; q < NR; q++)
            if (act[q]) {
                const double v[1] = {nrm[q]};
                partials_store_at<kBlock, 1>(v, partials + (long)(r0 + q) * b.pstride, xcd_block());
            }
}

// CG stage 4 for the NR rhs (the single-RHS arithmetic), |r_r|^2 partials
template <typename C, typename R, int CLOV, int LM, int NR>
__global__ __launch_bounds__(kBlock) void k_bm_hop4(Geom g, BatchT<R> b, VecsT<C> t, VecsT<C> T, VecsT<C> p,
                                                    VecsT<C> x, VecsT<C> rr, const C *__restrict__ U,
                                                    const double *__restrict__ st, double *__restrict__ partials,
                                                    int r0)
{
    const int tt = xcd_site(2 * g.Vh);
    bool act[NR];
    rhs_active<NR>(st, r0, act);
    double nrm[NR];
#pragma unroll
    for (int q = 0; q < NR; q++) nrm[q] = 0;
    if (tt >= 0) {
        const int i = tile_site(g, tt >> 1), hb = tt & 1;
        C acc[NR][6];
        hop_multi<LM, NR>(g, 0, i, hb, T.in + r0, U, (R)1, act, acc);
        const long Vh = g.Vh;
        const bool same = clover_shared<NR>(b.cle, r0);
        R d[6];
        C o[15];
        if (CLOV && same) clover_fetch(b.cle[r0], g.Vh, i, hb, d, o);
#pragma unroll
        for (int q = 0; q < NR; q++) {
            if (!act[q]) continue;
            const int r = r0 + q;
            const double *s = st + 8 * r;
            C tv[6], at[6];
            load_block_st<(LM >> 1) & 1>(t.in[r], g.Vh, i, hb, (R)-1, tv);
            if (CLOV) {
                if (!same) clover_fetch(b.cle[r], g.Vh, i, hb, d, o);
                clover_mul(d, o, tv, at);
            }
            const R alpha = (R)(s[B_RR] / s[B_PAP]), a = b.a[r];
            const C *pp = p.in[r];
            C *xx = x.out[r], *rv_ = rr.out[r];
#pragma unroll
            for (int k = 0; k < 6; k++) {
                C base = CLOV ? at[k] : tv[k];
                C kp = mk<C>(fmadd(a, acc[q][k].x, base.x), fmadd(a, acc[q][k].y, base.y));
                if (hb) kp = cneg(kp);
                const long e = (long)(6 * hb + k) * Vh + i;
                C pv = ld_st<(LM >> 1) & 1>(pp + e), xv = ld_st<(LM >> 1) & 1>(xx + e),
                  rv = ld_st<(LM >> 1) & 1>(rv_ + e);
                xv.x = fmadd(alpha, pv.x, xv.x); xv.y = fmadd(alpha, pv.y, xv.y);
                rv.x = fmadd(-alpha, kp.x, rv.x); rv.y = fmadd(-alpha, kp.y, rv.y);
                st_st<(LM >> 1) & 1>(xx + e, xv);
                st_st<(LM >> 1) & 1>(rv_ + e, rv);
                cnorm_acc(nrm[q], rv);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NR; q++)
        if (act[q]) {
            const double v[1] = {nrm[q]};
            partials_store_at<kBlock, 1>(v, partials + (long)(r0 + q) * b.pstride, xcd_block());
        }
}

// out = (FP32) (s * in); in FP64
__global__ void k_b_narrow(long n, double s, const double2 *__restrict__ in, float2 *__restrict__ out)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) out[t] = make_float2((float)(s * in[t].x), (float)(s * in[t].y));
}

// x += s * e (e FP32, x FP64)
__global__ void k_b_accum(long n, double s, const float2 *__restrict__ e, double2 *__restrict__ x)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) x[t] = make_double2(x[t].x + s * (double)e[t].x, x[t].y + s * (double)e[t].y);
}

}  // namespace

// launch the (C, R, CLOV, link mode) instance of a workgroup-per-rhs stencil kernel.  Link
// loads are never streaming here: the n workgroups of a site block read the same links, and the
// copy the first one brings into L2 is what the others reuse (on 32^3 x 64, 4
// right-hand sides: 0.85 of the single-RHS time per rhs, against 1.0 with streaming).
#define BLAUNCH(K, C, R, b, grid, block, shm, stream, ...)                                                   \
    do {                                                                                                  \
        const int lm_ = link_mode(ctx->g) & 1;                                                            \
        if ((b).clov[0]) {                                                                                \
            if (lm_ == 0) hipLaunchKernelGGL((K<C, R, 1, 0>), grid, block, shm, stream, __VA_ARGS__);       \
            else hipLaunchKernelGGL((K<C, R, 1, 1>), grid, block, shm, stream, __VA_ARGS__);                \
        } else {                                                                                          \
            if (lm_ == 0) hipLaunchKernelGGL((K<C, R, 0, 0>), grid, block, shm, stream, __VA_ARGS__);       \
            else hipLaunchKernelGGL((K<C, R, 0, 1>), grid, block, shm, stream, __VA_ARGS__);                \
        }                                                                                                 \
    } while (0)

// launch the (C, R, clover, link mode, NR) instance of a multi-rhs kernel for the nr (1..4)
// right-hand sides from r0, in the context's link mode (each link is read once per site here,
// so the FP64 links stream when the context streams them); the grid covers the sites once
// (XCD-aware order)
#define BM_LM_ONE(K, C, R, NR, LMV, grid, ...) \
    hipLaunchKernelGGL((K<C, R, 1, LMV, NR>), grid, dim3(kBlock), 0, ctx->stream, __VA_ARGS__)
#define BM_LM(K, C, R, NR, grid, ...)                                 \
    do {                                                            \
        switch (link_mode(ctx->g)) {                                \
        case 0: BM_LM_ONE(K, C, R, NR, 0, grid, __VA_ARGS__); break;  \
        case 1: BM_LM_ONE(K, C, R, NR, 1, grid, __VA_ARGS__); break;  \
        case 2: BM_LM_ONE(K, C, R, NR, 2, grid, __VA_ARGS__); break;  \
        default: BM_LM_ONE(K, C, R, NR, 3, grid, __VA_ARGS__); break; \
        }                                                           \
    } while (0)
#define BMLAUNCH(K, C, R, nr, grid, ...)                    \
    do {                                                    \
        switch (nr) {                                       \
        case 1: BM_LM(K, C, R, 1, grid, __VA_ARGS__); break; \
        case 2: BM_LM(K, C, R, 2, grid, __VA_ARGS__); break; \
        case 3: BM_LM(K, C, R, 3, grid, __VA_ARGS__); break; \
        default: BM_LM(K, C, R, 4, grid, __VA_ARGS__); break; \
        }                                                   \
    } while (0)
// right-hand sides per lane pair in the multi-rhs layout (at most 4): the context's choice, or
// by default 4 (measured fastest in FP32 and FP64)
static int multi_group(const pfmp_ctx *ctx)
{
    return ctx->batch_multi == 2 || ctx->batch_multi == 4 ? ctx->batch_multi : 4;
}

// the multi-rhs layout (each link load shared by up to 4 rhs in a lane) for clover batches
// unless switched off (pfmp_set_batch_layout)
template <typename R>
static bool use_multi(const pfmp_ctx *ctx, const BatchT<R> &b)
{
    return ctx->batch_multi && b.clov[0];
}

static int make_batch(pfmp_ctx *ctx, int nrhs, const int *ops, BatchT<double> &b, BatchT<float> &bf)
{
    if (nrhs <= 0 || nrhs > kMaxRhs || !ops) return set_err(ctx, PFMP_ERR_ARG, "batch: 1..8 right-hand sides");
    b.n = bf.n = nrhs;
    b.k = bf.k = nrhs;
    b.nsb = bf.nsb = nblocks(2L * ctx->g.Vh, kBlock);
    b.pstride = bf.pstride = ((b.nsb + 63) / 64) * 64;
    for (int r = 0; r < kMaxRhs; r++) {
        int op = r < nrhs ? ops[r] : ops[0];
        if (op < 0 || op >= PFMP_MAX_OPS || !ctx->ops[op].valid || !ctx->have_gauge)
            return set_err(ctx, PFMP_ERR_STATE, "batch: operator slot not configured");
        if (int rc0 = op_ready(ctx, op)) return rc0;
        const OpSlot &s = ctx->ops[op];
        b.clo[r] = s.clov[1];
        b.cle[r] = s.clov[0];
        b.a[r] = -s.kappa * s.kappa;
        bf.clo[r] = s.clovf[1];
        bf.cle[r] = s.clovf[0];
        bf.a[r] = (float)(-s.kappa * s.kappa);
        b.clov[r] = bf.clov[r] = s.csw != 0;
    }
    for (int r = 1; r < nrhs; r++)
        if (b.clov[r] != b.clov[0])
            return set_err(ctx, PFMP_ERR_ARG, "batch: all operators of a batch must be clover or all Wilson");
    return 0;
}

template <typename C>
static VecsT<C> vecs(int n, const void *const *in, void *const *out)
{
    VecsT<C> v{};
    for (int r = 0; r < n; r++) {
        v.in[r] = in ? (const C *)in[r] : nullptr;
        v.out[r] = out ? (C *)out[r] : nullptr;
    }
    return v;
}

// out_r = Khat_r in_r for all r: 4 launches (multi-rhs layout: 4 per group of 4 rhs)
template <typename C, typename R>
static int apply_batch(pfmp_ctx *ctx, const BatchT<R> &b, const C *U, int nrhs, const void *const *in,
                       void *const *out)
{
    const Geom &g = ctx->g;
    std::vector<void *> te(nrhs), to(nrhs);
    for (int r = 0; r < nrhs; r++) {
        te[r] = pool_get(ctx, 1000 + r);
        to[r] = pool_get(ctx, 1008 + r);
        if (!te[r] || !to[r]) return set_err(ctx, PFMP_ERR_OOM, "batch workspace");
    }
    const VecsT<C> in_to = vecs<C>(nrhs, in, to.data()), in_te = vecs<C>(nrhs, in, te.data());
    const VecsT<C> to_in = vecs<C>(nrhs, (const void *const *)to.data(), nullptr);
    const VecsT<C> te_to = vecs<C>(nrhs, (const void *const *)te.data(), to.data());
    const VecsT<C> te_out = vecs<C>(nrhs, (const void *const *)te.data(), out);
    // Mhat in -> te (stage 1 to to, stage 2 to te), then Mhat^dag te -> out
    if (use_multi(ctx, b)) {
        dim3 grid(op_nparts(g));
        const int mg = multi_group(ctx);
        for (int r0 = 0; r0 < nrhs; r0 += mg) {
            const int nr = std::min(mg, nrhs - r0);
            BMLAUNCH(k_bm_clovinv, C, R, nr, grid, g, b, in_to, U, (R)1, (R)1, (const double *)nullptr, r0);
            BMLAUNCH(k_bm_xpay, C, R, nr, grid, g, b, in_te, to_in, U, (R)1, (const double *)nullptr,
                     (double *)nullptr, r0);
            BMLAUNCH(k_bm_clovinv, C, R, nr, grid, g, b, te_to, U, (R)-1, (R)1, (const double *)nullptr, r0);
            BMLAUNCH(k_bm_xpay, C, R, nr, grid, g, b, te_out, to_in, U, (R)-1, (const double *)nullptr,
                     (double *)nullptr, r0);
        }
    } else {
        dim3 grid(((b.nsb * nrhs + 7) / 8) * 8), block(kBlock);
        BLAUNCH(k_b_clovinv, C, R, b, grid, block, 0, ctx->stream, g, b, in_to, U, (R)1, (R)1, nullptr);
        BLAUNCH(k_b_xpay, C, R, b, grid, block, 0, ctx->stream, g, b, in_te, to_in, U, (R)1, nullptr, nullptr);
        BLAUNCH(k_b_clovinv, C, R, b, grid, block, 0, ctx->stream, g, b, te_to, U, (R)-1, (R)1, nullptr);
        BLAUNCH(k_b_xpay, C, R, b, grid, block, 0, ctx->stream, g, b, te_out, to_in, U, (R)-1, nullptr, nullptr);
    }
    LAUNCHCHK(ctx);
    return 0;
}

extern "C" int pfmp_apply_MdagM_batch(pfmp_ctx *ctx, int nrhs, const int *ops, const void *const *in,
                                      void *const *out, int prec)
{
    if (!ctx) return PFMP_ERR_ARG;
    BatchT<double> b;
    BatchT<float> bf;
    int rc = make_batch(ctx, nrhs, ops, b, bf);
    if (rc) return rc;
    if (!in || !out) return set_err(ctx, PFMP_ERR_ARG, "batch: null buffers");
    for (int r = 0; r < nrhs; r++)
        if (!in[r] || !out[r]) return set_err(ctx, PFMP_ERR_ARG, "batch: null buffer");
    if (prec == PFMP_F64) return apply_batch<double2, double>(ctx, b, ctx->U, nrhs, in, out);
    if (prec == PFMP_F32) {
        if ((rc = gauge_f32_ready(ctx))) return rc;
        return apply_batch<float2, float>(ctx, bf, ctx->Uf, nrhs, in, out);
    }
    return set_err(ctx, PFMP_ERR_ARG, "apply_MdagM_batch: FP64 or FP32 fields");
}

extern "C" int pfmp_set_batch_layout(pfmp_ctx *ctx, int multi)
{
    if (!ctx) return PFMP_ERR_ARG;
    if (multi != 0 && multi != 1 && multi != 2 && multi != 4)
        return set_err(ctx, PFMP_ERR_ARG, "batch layout: 0, 1, 2 or 4");
    ctx->batch_multi = multi;
    return 0;
}

// Batched CG in the field type C from x_r = 0: rhs r runs until its recursive |r|^2 <=
// thr[r] (or it is skipped: skip[r]), at most maxiter iterations; iters[r] filled.
// rr0[r] = |b_r|^2.  Work buffers come from the pool at base (4 per rhs).
template <typename C, typename R>
static int batch_cg_core(pfmp_ctx *ctx, const BatchT<R> &b, const void *const *b_, void *const *x_,
                         const double *rr0, const double *thr, const bool *skip, int maxiter, int check_every,
                         int base, int *iters, double *done)
{
    const Geom &g = ctx->g;
    const int nrhs = b.n;
    const size_t vb = sizeof(R) * spinor_reals(g);
    const long n = 12L * g.Vh;
    std::vector<void *> Rv(nrhs), P(nrhs), T1(nrhs), T2(nrhs);
    for (int r = 0; r < nrhs; r++) {
        Rv[r] = pool_get(ctx, base + r);
        P[r] = pool_get(ctx, base + 8 + r);
        T1[r] = pool_get(ctx, base + 16 + r);
        T2[r] = pool_get(ctx, base + 24 + r);
        if (!Rv[r] || !P[r] || !T1[r] || !T2[r]) return set_err(ctx, PFMP_ERR_OOM, "batch workspace");
        HIPCHK(ctx, hipMemsetAsync(x_[r], 0, vb, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(Rv[r], b_[r], vb, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(P[r], b_[r], vb, hipMemcpyDeviceToDevice, ctx->stream));
    }
    const int ngrid = ((b.nsb * nrhs + 7) / 8) * 8;
    double *part_a = (double *)ws_alloc(ctx, sizeof(double) * b.pstride * b.k, 9);
    double *part_b = (double *)ws_alloc(ctx, sizeof(double) * b.pstride * b.k, 10);
    if (!part_a || !part_b) return set_err(ctx, PFMP_ERR_OOM, "batch workspace");
    double *sc = ctx->scal + kBatchBase;
    std::vector<double> init(8 * kMaxRhs, 0.0);
    for (int r = 0; r < nrhs; r++) {
        init[8 * r + B_RR] = rr0[r];
        init[8 * r + B_THR] = thr[r];
        init[8 * r + B_DONE] = (rr0[r] == 0 || (skip && skip[r])) ? 1 : 0;
        init[8 * r + B_MAXIT] = maxiter;
    }
    HIPCHK(ctx, hipMemcpyAsync(sc, init.data(), sizeof(double) * 8 * kMaxRhs, hipMemcpyHostToDevice, ctx->stream));
    dim3 grid(ngrid), block(kBlock);
    const VecsT<C> vP = vecs<C>(nrhs, (const void *const *)P.data(), P.data());
    const VecsT<C> vT1 = vecs<C>(nrhs, (const void *const *)T1.data(), T1.data());
    const VecsT<C> vT2 = vecs<C>(nrhs, (const void *const *)T2.data(), T2.data());
    const VecsT<C> vR = vecs<C>(nrhs, (const void *const *)Rv.data(), Rv.data());
    const VecsT<C> vX = vecs<C>(nrhs, nullptr, x_);
    // stage buffers: T2 <- A^-1 D_oe p ; T1 <- Mhat p ; T2 <- A^-1 D_oe g5 T1
    const VecsT<C> p_to_T2 = vecs<C>(nrhs, (const void *const *)P.data(), T2.data());
    const VecsT<C> p_to_T1 = vecs<C>(nrhs, (const void *const *)P.data(), T1.data());
    const VecsT<C> T1_to_T2 = vecs<C>(nrhs, (const void *const *)T1.data(), T2.data());
    const C *U = sizeof(R) == 8 ? (const C *)ctx->U : (const C *)ctx->Uf;
    int chunk = check_every > 0 ? check_every : 25;
    const bool multi = use_multi(ctx, b);
    const int mg = multi_group(ctx);
    dim3 gridm(op_nparts(g));
    // one iteration for all rhs: 7 launches with fixed arguments (4 more per further group of
    // 4 rhs in the multi-rhs layout), replayed as a graph; each rhs takes the single-RHS CG's
    // steps in its arithmetic and summation order
    auto iteration = [&]() -> int {
        if (multi) {
            for (int r0 = 0; r0 < nrhs; r0 += mg)
                BMLAUNCH(k_bm_clovinv, C, R, std::min(mg, nrhs - r0), gridm, g, b, p_to_T2, U, (R)1, (R)1,
                         (const double *)sc, r0);
            for (int r0 = 0; r0 < nrhs; r0 += mg)
                BMLAUNCH(k_bm_xpay, C, R, std::min(mg, nrhs - r0), gridm, g, b, p_to_T1, vT2, U, (R)1,
                         (const double *)sc, part_a, r0);
        } else {
            BLAUNCH(k_b_clovinv, C, R, b, grid, block, 0, ctx->stream, g, b, p_to_T2, U, (R)1, (R)1, sc);
            BLAUNCH(k_b_xpay, C, R, b, grid, block, 0, ctx->stream, g, b, p_to_T1, vT2, U, (R)1, sc, part_a);
        }
        hipLaunchKernelGGL(k_b_pap, dim3(1), dim3(kFinishThreads), 0, ctx->stream, part_a, b.nsb, b.pstride, nrhs,
                           sc);
        if (multi) {
            for (int r0 = 0; r0 < nrhs; r0 += mg)
                BMLAUNCH(k_bm_clovinv, C, R, std::min(mg, nrhs - r0), gridm, g, b, T1_to_T2, U, (R)-1, (R)1,
                         (const double *)sc, r0);
            for (int r0 = 0; r0 < nrhs; r0 += mg)
                BMLAUNCH(k_bm_hop4, C, R, std::min(mg, nrhs - r0), gridm, g, b, vT1, vT2, vP, vX, vR, U,
                         (const double *)sc, part_b, r0);
        } else {
            BLAUNCH(k_b_clovinv, C, R, b, grid, block, 0, ctx->stream, g, b, T1_to_T2, U, (R)-1, (R)1, sc);
            BLAUNCH(k_b_hop4, C, R, b, grid, block, 0, ctx->stream, g, b, vT1, vT2, vP, vX, vR, U, sc, part_b);
        }
        hipLaunchKernelGGL(k_b_beta, dim3(1), dim3(kFinishThreads), 0, ctx->stream, part_b, b.nsb, b.pstride, nrhs,
                           sc);
        hipLaunchKernelGGL((k_b_update_p<C>), dim3(nblocks(n * nrhs, 256)), dim3(256), 0, ctx->stream, g, nrhs, vR,
                           vP, sc);
        LAUNCHCHK(ctx);
        return 0;
    };
    std::vector<uint64_t> key;
    key_add(key, 5);   // batched CG iteration
    key_add(key, (int)sizeof(R));
    key_geom(key, g);
    key_add(key, nrhs);
    for (int r = 0; r < nrhs; r++) {
        for (const void *ptr : {(const void *)P[r], (const void *)T1[r], (const void *)T2[r], (const void *)Rv[r],
                                (const void *)x_[r], (const void *)b.clo[r], (const void *)b.cle[r]})
            key_add(key, ptr);
        key_add(key, b.a[r]);
    }
    for (const void *ptr : {(const void *)part_a, (const void *)part_b, (const void *)sc, (const void *)U})
        key_add(key, ptr);
    key_add(key, b.clov[0]);
    key_add(key, (int)multi);
    key_add(key, mg);
    for (;;) {
        bool all = true;
        for (int r = 0; r < nrhs; r++) all = all && init[8 * r + B_DONE] != 0;
        if (all) break;
        int rc;
        if ((rc = graph_run(ctx, key, chunk, iteration))) return rc;
        HIPCHK(ctx, hipMemcpyAsync(ctx->red_host, sc, sizeof(double) * 8 * kMaxRhs, hipMemcpyDeviceToHost,
                                   ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        for (int r = 0; r < nrhs; r++) {
            init[8 * r + B_DONE] = ctx->red_host[8 * r + B_DONE];
            init[8 * r + B_ITER] = ctx->red_host[8 * r + B_ITER];
        }
    }
    for (int r = 0; r < nrhs; r++) {
        iters[r] = (int)init[8 * r + B_ITER];
        done[r] = init[8 * r + B_DONE];
    }
    return 0;
}

// FP64 |b - Khat_op x|^2
static int residual64(pfmp_ctx *ctx, int op, const double2 *b, const double2 *x, double2 *res, double *rr)
{
    const Geom &g = ctx->g;
    const size_t vb = sizeof(double) * spinor_reals(g);
    double2 *Kx = (double2 *)ws_alloc(ctx, vb, 8), *te = (double2 *)ws_alloc(ctx, vb, 6),
            *to = (double2 *)ws_alloc(ctx, vb, 7);
    if (!Kx || !te || !to) return set_err(ctx, PFMP_ERR_OOM, "batch workspace");
    int rc;
    if ((rc = op_apply_K(ctx, op, x, Kx, te, to, nullptr))) return rc;
    double one[2] = {1, 0}, mone[2] = {-1, 0};
    HIPCHK(ctx, hipMemcpyAsync(res, b, vb, hipMemcpyDeviceToDevice, ctx->stream));
    if ((rc = pfmp_axpby(ctx, mone, Kx, one, res))) return rc;
    if ((rc = launch_norm2(ctx, res, 12L * g.Vh, ctx->red))) return rc;
    return red_finish(ctx, ctx->red, ctx->nblk_red, 1, rr);
}

extern "C" int pfmp_cg_solve_batch(pfmp_ctx *ctx, int nrhs, const int *ops, const void *const *b_, void *const *x_,
                                   const pfmp_solver_params *prm, pfmp_solver_stats *st)
{
    if (!ctx) return PFMP_ERR_ARG;
    BatchT<double> b;
    BatchT<float> bf;
    int rc = make_batch(ctx, nrhs, ops, b, bf);
    if (rc) return rc;
    if (!b_ || !x_ || !prm || !(prm->tol > 0) || prm->maxiter <= 0)
        return set_err(ctx, PFMP_ERR_ARG, "cg_solve_batch: bad arguments");
    if (prm->prec != PFMP_F64 && prm->prec != PFMP_F32 && prm->prec != PFMP_F16)
        return set_err(ctx, PFMP_ERR_ARG, "cg_solve_batch: precision");
    for (int r = 0; r < nrhs; r++)
        if (!b_[r] || !x_[r]) return set_err(ctx, PFMP_ERR_ARG, "cg_solve_batch: null buffer");
    if (prm->prec != PFMP_F64 && (rc = gauge_f32_ready(ctx))) return rc;
    auto t0 = std::chrono::steady_clock::now();
    const Geom &g = ctx->g;
    const size_t vb = sizeof(double) * spinor_reals(g);
    const long n = 12L * g.Vh;
    std::vector<double> bb(nrhs), thr(nrhs), res(nrhs, 0.0), done(nrhs, 0.0);
    std::vector<int> its(nrhs, 0), total(nrhs, 0), outer(nrhs, 0);
    for (int r = 0; r < nrhs; r++) {
        if ((rc = launch_norm2(ctx, (const double2 *)b_[r], n, ctx->red))) return rc;
        if ((rc = red_finish(ctx, ctx->red, ctx->nblk_red, 1, &bb[r]))) return rc;
        thr[r] = prm->tol * prm->tol * bb[r];
    }
    int worst_rc = 0;
    std::vector<double2 *> rv(nrhs);
    for (int r = 0; r < nrhs; r++)
        if (!(rv[r] = pool_get(ctx, 1032 + r))) return set_err(ctx, PFMP_ERR_OOM, "batch workspace");
    if (prm->prec == PFMP_F64) {
        if ((rc = batch_cg_core<double2, double>(ctx, b, b_, x_, bb.data(), thr.data(), nullptr, prm->maxiter,
                                                 prm->check_every, 1000, its.data(), done.data())))
            return rc;
        for (int r = 0; r < nrhs; r++) {
            double rr;
            if ((rc = residual64(ctx, ops[r], (const double2 *)b_[r], (const double2 *)x_[r], rv[r], &rr))) return rc;
            res[r] = bb[r] > 0 ? std::sqrt(rr / bb[r]) : 0;
            total[r] = its[r];
            if (done[r] == 2 && !(res[r] <= prm->tol)) worst_rc = PFMP_ERR_NOCONV;
        }
    } else {
        // defect correction: FP64 residuals and solution, FP32 batched inner solves
        std::vector<void *> r32(nrhs), e32(nrhs);
        for (int r = 0; r < nrhs; r++) {
            r32[r] = pool_get(ctx, 1040 + r);
            e32[r] = pool_get(ctx, 1048 + r);
            if (!r32[r] || !e32[r]) return set_err(ctx, PFMP_ERR_OOM, "batch workspace");
            HIPCHK(ctx, hipMemsetAsync(x_[r], 0, vb, ctx->stream));
            HIPCHK(ctx, hipMemcpyAsync(rv[r], b_[r], vb, hipMemcpyDeviceToDevice, ctx->stream));
        }
        std::vector<double> rr(bb), one(nrhs, 1.0), ithr(nrhs);
        std::vector<bool> conv(nrhs);
        for (;;) {
            bool all = true;
            for (int r = 0; r < nrhs; r++) {
                conv[r] = rr[r] <= thr[r];
                all = all && conv[r];
            }
            if (all) break;
            bool spent = false;
            for (int r = 0; r < nrhs; r++) spent = spent || (!conv[r] && total[r] >= prm->maxiter);
            if (spent) {
                worst_rc = PFMP_ERR_NOCONV;
                break;
            }
            bool skip[kMaxRhs] = {};
            int budget = prm->maxiter;
            for (int r = 0; r < nrhs; r++) {
                skip[r] = conv[r];
                // relative reduction asked of this pass, no tighter than FP32 reaches
                const double need = 0.5 * prm->tol * std::sqrt(bb[r] / rr[r]);
                ithr[r] = std::max(need, 2e-6) * std::max(need, 2e-6);
                if (!conv[r]) budget = std::min(budget, prm->maxiter - total[r]);
                hipLaunchKernelGGL(k_b_narrow, dim3(nblocks(n, 256)), dim3(256), 0, ctx->stream, n,
                                   conv[r] ? 0.0 : 1.0 / std::sqrt(rr[r]), rv[r], (float2 *)r32[r]);
            }
            LAUNCHCHK(ctx);
            if ((rc = batch_cg_core<float2, float>(ctx, bf, (const void *const *)r32.data(), e32.data(), one.data(),
                                                   ithr.data(), skip, std::max(budget, 1), prm->check_every, 1056,
                                                   its.data(), done.data())))
                return rc;
            for (int r = 0; r < nrhs; r++) {
                if (conv[r]) continue;
                total[r] += its[r];
                outer[r]++;
                hipLaunchKernelGGL(k_b_accum, dim3(nblocks(n, 256)), dim3(256), 0, ctx->stream, n, std::sqrt(rr[r]),
                                   (const float2 *)e32[r], (double2 *)x_[r]);
                LAUNCHCHK(ctx);
                if ((rc = residual64(ctx, ops[r], (const double2 *)b_[r], (const double2 *)x_[r], rv[r], &rr[r])))
                    return rc;
            }
        }
        for (int r = 0; r < nrhs; r++) res[r] = bb[r] > 0 ? std::sqrt(rr[r] / bb[r]) : 0;
    }
    auto t1 = std::chrono::steady_clock::now();
    if (st)
        for (int r = 0; r < nrhs; r++) {
            st[r] = pfmp_solver_stats{};
            st[r].iters = total[r];
            st[r].reliable_updates = outer[r];
            st[r].true_res = res[r];
            st[r].kmults = total[r] + (prm->prec == PFMP_F64 ? 1 : outer[r]);
            st[r].seconds = std::chrono::duration<double>(t1 - t0).count();
        }
    if (worst_rc) return set_err(ctx, worst_rc, "cg_solve_batch: maxiter reached");
    return 0;
}
