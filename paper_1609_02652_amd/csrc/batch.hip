// batch.hip -- multi-RHS operator and CG: k right-hand sides, each with its own
// operator slot (kappa, clover), in one launch per stage.
//
// Each workgroup serves one right-hand side (so every pointer and scalar of the rhs is
// uniform in the workgroup) with the two-lanes-per-site kernels of the single-RHS
// operator.  The n workgroups that cover the same block of sites for the n right-hand
// sides are consecutive in the XCD-aware block order, so they run together on one XCD
// and every link is fetched once into its L2 for all n.  Per-rhs CG scalars and
// convergence flags live on the device; a converged rhs stops touching memory.
// Reductions: one FP64 partial per workgroup (indexed site block * n + rhs), fixed order.
#include <chrono>
#include <cmath>

#include "hop.h"

namespace {

constexpr int kMaxRhs = 8;
enum { B_RR = 0, B_THR, B_PAP, B_ALPHA, B_BETA, B_ITER, B_DONE, B_MAXIT, B_NSLOT = 8 };
constexpr int kBatchBase = 5120;   // per-rhs scalar records at ctx->scal + kBatchBase + 8 r

struct Batch {
    int k;                          // stride of the partials (= n)
    int n;                          // right-hand sides
    int nsb;                        // site blocks (two lanes per site, kBlock lanes per block)
    const double *clo[kMaxRhs];     // A_oo^-1 of each rhs's operator
    const double *cle[kMaxRhs];     // A_ee
    double a[kMaxRhs];              // -kappa^2
    int clov[kMaxRhs];
};

struct Vecs {
    const double2 *in[kMaxRhs];
    double2 *out[kMaxRhs];
};

// logical workgroup lb = site block * n + rhs (XCD-aware order); false past the end
__device__ __forceinline__ bool item(const Geom &g, const Batch &b, int *lb, int *site, int *r, int *hb)
{
    const int nb = gridDim.x, bi = blockIdx.x;
    const int per = (nb + 7) >> 3;
    *lb = (bi & 7) * per + (bi >> 3);
    if (*lb >= b.nsb * b.n) return false;
    *r = *lb % b.n;
    const int t = (*lb / b.n) * blockDim.x + threadIdx.x;
    if (t >= 2 * g.Vh) return false;
    *site = tile_site(g, t >> 1);
    *hb = t & 1;
    return true;
}

// one FP64 partial per logical workgroup (every thread of the block calls this)
__device__ __forceinline__ void batch_partial(double v, int lb, int nlb, double *partials)
{
    __shared__ double sh[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0 && lb < nlb) {
        double s = 0;
        for (int q = 0; q < kBlock / 64; q++) s += sh[q];
        partials[lb] = s;
    }
}

// out_r = [g5] A_oo^-1 D_oe [g5] in_r
template <int CLOV, int LM>
__global__ __launch_bounds__(kBlock) void k_b_clovinv(Geom g, Batch b, Vecs v, const double2 *__restrict__ U,
                                                      double gin, double gout, const double *__restrict__ st)
{
    int lb, i, r, hb;
    if (!item(g, b, &lb, &i, &r, &hb)) return;
    if (st && st[8 * r + B_DONE] != 0) return;
    double2 blk[6];
    hop_pair<LM, double2>(g, 1, i, hb, v.in[r], U, gin, blk);
    if (CLOV) {
        double2 t[6];
        clover_block<double, double2>(b.clo[r], g.Vh, i, hb, blk, t);
        store_block(v.out[r], g.Vh, i, hb, gout, t);
    } else {
        store_block(v.out[r], g.Vh, i, hb, gout, blk);
    }
}

// out_r = [g5] (A_ee [g5] x_r + a_r D_eo t_r), |out_r|^2 partials
template <int CLOV, int LM>
__global__ __launch_bounds__(kBlock) void k_b_xpay(Geom g, Batch b, Vecs x, Vecs t, const double2 *__restrict__ U,
                                                   double gs, const double *__restrict__ st,
                                                   double *__restrict__ partials)
{
    int lb = 0, i = 0, r = 0, hb = 0;
    bool ok = item(g, b, &lb, &i, &r, &hb);
    if (ok && st && st[8 * r + B_DONE] != 0) ok = false;
    double nrm = 0;
    if (ok) {
        double2 acc[6], xv[6], ax[6];
        hop_pair<LM, double2>(g, 0, i, hb, t.in[r], U, 1.0, acc);
        load_block(x.in[r], g.Vh, i, hb, gs, xv);
        if (CLOV) clover_block<double, double2>(b.cle[r], g.Vh, i, hb, xv, ax);
        const double a = b.a[r];
#pragma unroll
        for (int k = 0; k < 6; k++) {
            double2 base = CLOV ? ax[k] : xv[k];
            acc[k] = make_double2(base.x + a * acc[k].x, base.y + a * acc[k].y);
            nrm += acc[k].x * acc[k].x + acc[k].y * acc[k].y;
        }
        store_block(x.out[r], g.Vh, i, hb, gs, acc);
    }
    if (partials) batch_partial(nrm, lb, b.nsb * b.n, partials);
}

// CG stage 4: Kp_r from t_r and T'_r; x_r += alpha_r p_r; r_r -= alpha_r Kp_r; |r_r|^2 partials
template <int CLOV, int LM>
__global__ __launch_bounds__(kBlock) void k_b_hop4(Geom g, Batch b, Vecs t, Vecs T, Vecs p, Vecs x, Vecs rr,
                                                   const double2 *__restrict__ U, const double *__restrict__ st,
                                                   double *__restrict__ partials)
{
    int lb = 0, i = 0, r = 0, hb = 0;
    bool ok = item(g, b, &lb, &i, &r, &hb);
    if (ok && st[8 * r + B_DONE] != 0) ok = false;
    double nrm = 0;
    if (ok) {
        double2 acc[6], tv[6], at[6];
        hop_pair<LM, double2>(g, 0, i, hb, T.in[r], U, 1.0, acc);
        load_block(t.in[r], g.Vh, i, hb, -1.0, tv);
        if (CLOV) clover_block<double, double2>(b.cle[r], g.Vh, i, hb, tv, at);
        const double alpha = st[8 * r + B_ALPHA], a = b.a[r];
        const long Vh = g.Vh;
        const double2 *pp = p.in[r];
        double2 *xx = x.out[r], *rv_ = rr.out[r];
#pragma unroll
        for (int k = 0; k < 6; k++) {
            double2 base = CLOV ? at[k] : tv[k];
            double2 kp = make_double2(base.x + a * acc[k].x, base.y + a * acc[k].y);
            if (hb) kp = cneg(kp);
            const long e = (long)(6 * hb + k) * Vh + i;
            double2 pv = pp[e], xv = xx[e], rv = rv_[e];
            xv.x += alpha * pv.x; xv.y += alpha * pv.y;
            rv.x -= alpha * kp.x; rv.y -= alpha * kp.y;
            xx[e] = xv;
            rv_[e] = rv;
            nrm += rv.x * rv.x + rv.y * rv.y;
        }
    }
    batch_partial(nrm, lb, b.nsb * b.n, partials);
}

__device__ __forceinline__ double rhs_total(const double *__restrict__ partials, int nparts, int k, int r)
{
    __shared__ double sh[kRedBlock / 64];
    double s = 0;
    for (int q = threadIdx.x; q < nparts; q += blockDim.x) s += partials[q * k + r];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    double tot = 0;
    for (int q = 0; q < kRedBlock / 64; q++) tot += sh[q];
    __syncthreads();
    return tot;
}

__global__ __launch_bounds__(kRedBlock) void k_b_alpha(const double *__restrict__ partials, int nparts, int k, int n,
                                                       double *__restrict__ st)
{
    for (int r = 0; r < n; r++) {
        if (st[8 * r + B_DONE] != 0) continue;
        double pap = rhs_total(partials, nparts, k, r);
        if (threadIdx.x == 0) {
            st[8 * r + B_PAP] = pap;
            st[8 * r + B_ALPHA] = st[8 * r + B_RR] / pap;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kRedBlock) void k_b_beta(const double *__restrict__ partials, int nparts, int k, int n,
                                                      double *__restrict__ st)
{
    for (int r = 0; r < n; r++) {
        double *s = st + 8 * r;
        if (s[B_DONE] != 0) continue;
        double rr = rhs_total(partials, nparts, k, r);
        if (threadIdx.x == 0) {
            s[B_BETA] = rr / s[B_RR];
            s[B_RR] = rr;
            s[B_ITER] += 1;
            s[B_DONE] = rr <= s[B_THR] ? 1 : (s[B_ITER] >= s[B_MAXIT] ? 2 : 0);
        }
        __syncthreads();
    }
}

// p_r = r_r + beta_r p_r for the right-hand sides still running
__global__ void k_b_update_p(Geom g, Batch b, Vecs rr, Vecs p, const double *__restrict__ st)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    long n = 12L * g.Vh;
    int r = (int)(t / n);
    long e = t - (long)r * n;
    if (r >= b.n || st[8 * r + B_DONE] != 0) return;
    double beta = st[8 * r + B_BETA];
    double2 rv = rr.in[r][e], pv = p.out[r][e];
    p.out[r][e] = make_double2(rv.x + beta * pv.x, rv.y + beta * pv.y);
}

}  // namespace

// launch the (CLOV, link mode) instance of a batch stencil kernel.  Link loads are never
// streaming here: the n workgroups of a site block read the same links, and the copy the
// first one brings into L2 is what the others reuse (on 32^3 x 64, 4 right-hand sides:
// 0.85 of the single-RHS time per rhs, against 1.0 with streaming loads).
#define BLAUNCH(K, grid, block, shm, stream, ...)                                                        \
    do {                                                                                              \
        const int lm_ = link_mode(ctx->g) & 1;                                                        \
        if (b.clov[0]) {                                                                              \
            if (lm_ == 0) hipLaunchKernelGGL((K<1, 0>), grid, block, shm, stream, __VA_ARGS__);         \
            else hipLaunchKernelGGL((K<1, 1>), grid, block, shm, stream, __VA_ARGS__);                  \
        } else {                                                                                      \
            if (lm_ == 0) hipLaunchKernelGGL((K<0, 0>), grid, block, shm, stream, __VA_ARGS__);         \
            else hipLaunchKernelGGL((K<0, 1>), grid, block, shm, stream, __VA_ARGS__);                  \
        }                                                                                             \
    } while (0)

static int make_batch(pfmp_ctx *ctx, int nrhs, const int *ops, Batch &b)
{
    if (nrhs <= 0 || nrhs > kMaxRhs || !ops) return set_err(ctx, PFMP_ERR_ARG, "batch: 1..8 right-hand sides");
    b.n = nrhs;
    b.k = nrhs;
    b.nsb = nblocks(2L * ctx->g.Vh, kBlock);
    for (int r = 0; r < kMaxRhs; r++) {
        int op = r < nrhs ? ops[r] : ops[0];
        if (op < 0 || op >= PFMP_MAX_OPS || !ctx->ops[op].valid || !ctx->have_gauge)
            return set_err(ctx, PFMP_ERR_STATE, "batch: operator slot not configured");
        if (int rc0 = op_ready(ctx, op)) return rc0;
        const OpSlot &s = ctx->ops[op];
        b.clo[r] = s.clov[1];
        b.cle[r] = s.clov[0];
        b.a[r] = -s.kappa * s.kappa;
        b.clov[r] = s.csw != 0;
    }
    for (int r = 1; r < nrhs; r++)
        if (b.clov[r] != b.clov[0])
            return set_err(ctx, PFMP_ERR_ARG, "batch: all operators of a batch must be clover or all Wilson");
    return 0;
}

static Vecs vecs(int n, const void *const *in, void *const *out)
{
    Vecs v{};
    for (int r = 0; r < n; r++) {
        v.in[r] = in ? (const double2 *)in[r] : nullptr;
        v.out[r] = out ? (double2 *)out[r] : nullptr;
    }
    return v;
}

// out_r = Khat_r in_r for all r: 4 launches regardless of the number of rhs
extern "C" int pfmp_apply_MdagM_batch(pfmp_ctx *ctx, int nrhs, const int *ops, const void *const *in,
                                      void *const *out)
{
    if (!ctx) return PFMP_ERR_ARG;
    Batch b;
    int rc = make_batch(ctx, nrhs, ops, b);
    if (rc) return rc;
    if (!in || !out) return set_err(ctx, PFMP_ERR_ARG, "batch: null buffers");
    for (int r = 0; r < nrhs; r++)
        if (!in[r] || !out[r]) return set_err(ctx, PFMP_ERR_ARG, "batch: null buffer");
    const Geom &g = ctx->g;
    std::vector<void *> te(nrhs), to(nrhs);
    for (int r = 0; r < nrhs; r++) {
        te[r] = pool_get(ctx, 1000 + r);
        to[r] = pool_get(ctx, 1008 + r);
        if (!te[r] || !to[r]) return set_err(ctx, PFMP_ERR_OOM, "batch workspace");
    }
    dim3 grid(((b.nsb * nrhs + 7) / 8) * 8), block(kBlock);
    // Mhat in -> te (stage 1 to to, stage 2 to te), then Mhat^dag te -> out
    BLAUNCH(k_b_clovinv, grid, block, 0, ctx->stream, g, b, vecs(nrhs, in, to.data()), ctx->U, 1.0, 1.0,
                       nullptr);
    BLAUNCH(k_b_xpay, grid, block, 0, ctx->stream, g, b, vecs(nrhs, in, te.data()),
                       vecs(nrhs, (const void *const *)to.data(), nullptr), ctx->U, 1.0, nullptr, nullptr);
    BLAUNCH(k_b_clovinv, grid, block, 0, ctx->stream, g, b,
                       vecs(nrhs, (const void *const *)te.data(), to.data()), ctx->U, -1.0, 1.0, nullptr);
    BLAUNCH(k_b_xpay, grid, block, 0, ctx->stream, g, b, vecs(nrhs, (const void *const *)te.data(), out),
                       vecs(nrhs, (const void *const *)to.data(), nullptr), ctx->U, -1.0, nullptr, nullptr);
    LAUNCHCHK(ctx);
    return 0;
}

extern "C" int pfmp_cg_solve_batch(pfmp_ctx *ctx, int nrhs, const int *ops, const void *const *b_, void *const *x_,
                                   const pfmp_solver_params *prm, pfmp_solver_stats *st)
{
    if (!ctx) return PFMP_ERR_ARG;
    Batch b;
    int rc = make_batch(ctx, nrhs, ops, b);
    if (rc) return rc;
    if (!b_ || !x_ || !prm || !(prm->tol > 0) || prm->maxiter <= 0)
        return set_err(ctx, PFMP_ERR_ARG, "cg_solve_batch: bad arguments");
    if (prm->prec != PFMP_F64) return set_err(ctx, PFMP_ERR_ARG, "cg_solve_batch: FP64 only");
    for (int r = 0; r < nrhs; r++)
        if (!b_[r] || !x_[r]) return set_err(ctx, PFMP_ERR_ARG, "cg_solve_batch: null buffer");
    auto t0 = std::chrono::steady_clock::now();
    const Geom &g = ctx->g;
    const size_t vb = sizeof(double) * spinor_reals(g);
    const long n = 12L * g.Vh;
    std::vector<void *> R(nrhs), P(nrhs), T1(nrhs), T2(nrhs);
    for (int r = 0; r < nrhs; r++) {
        R[r] = pool_get(ctx, 1016 + r);
        P[r] = pool_get(ctx, 1024 + r);
        T1[r] = pool_get(ctx, 1000 + r);
        T2[r] = pool_get(ctx, 1008 + r);
        if (!R[r] || !P[r] || !T1[r] || !T2[r]) return set_err(ctx, PFMP_ERR_OOM, "batch workspace");
        HIPCHK(ctx, hipMemsetAsync(x_[r], 0, vb, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(R[r], b_[r], vb, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(P[r], b_[r], vb, hipMemcpyDeviceToDevice, ctx->stream));
    }
    const int nb = b.nsb;   // partials per rhs
    const int ngrid = ((b.nsb * nrhs + 7) / 8) * 8;
    double *part_a = (double *)ws_alloc(ctx, sizeof(double) * (nb + 64) * b.k, 9);
    double *part_b = (double *)ws_alloc(ctx, sizeof(double) * (nb + 64) * b.k, 10);
    if (!part_a || !part_b) return set_err(ctx, PFMP_ERR_OOM, "batch workspace");
    double *sc = ctx->scal + kBatchBase;
    std::vector<double> bb(nrhs);
    for (int r = 0; r < nrhs; r++) {
        if ((rc = launch_norm2(ctx, (const double2 *)b_[r], n, ctx->red))) return rc;
        if ((rc = red_finish(ctx, ctx->red, ctx->nblk_red, 1, &bb[r]))) return rc;
    }
    std::vector<double> init(8 * kMaxRhs, 0.0);
    for (int r = 0; r < nrhs; r++) {
        init[8 * r + B_RR] = bb[r];
        init[8 * r + B_THR] = prm->tol * prm->tol * bb[r];
        init[8 * r + B_DONE] = bb[r] == 0 ? 1 : 0;
        init[8 * r + B_MAXIT] = prm->maxiter;
    }
    HIPCHK(ctx, hipMemcpyAsync(sc, init.data(), sizeof(double) * 8 * kMaxRhs, hipMemcpyHostToDevice, ctx->stream));
    dim3 grid(ngrid), block(kBlock);
    const Vecs vP = vecs(nrhs, (const void *const *)P.data(), P.data());
    const Vecs vT1 = vecs(nrhs, (const void *const *)T1.data(), T1.data());
    const Vecs vT2 = vecs(nrhs, (const void *const *)T2.data(), T2.data());
    const Vecs vR = vecs(nrhs, (const void *const *)R.data(), R.data());
    const Vecs vX = vecs(nrhs, nullptr, x_);
    // stage buffers: T2 <- A^-1 D_oe p ; T1 <- Mhat p ; T2 <- A^-1 D_oe g5 T1
    const Vecs p_to_T2 = vecs(nrhs, (const void *const *)P.data(), T2.data());
    const Vecs p_to_T1 = vecs(nrhs, (const void *const *)P.data(), T1.data());
    const Vecs T1_to_T2 = vecs(nrhs, (const void *const *)T1.data(), T2.data());
    int chunk = prm->check_every > 0 ? prm->check_every : 25;
    std::vector<double> h(8 * kMaxRhs);
    // one iteration for all rhs: 7 launches with fixed arguments, replayed as a graph
    auto iteration = [&]() -> int {
        BLAUNCH(k_b_clovinv, grid, block, 0, ctx->stream, g, b, p_to_T2, ctx->U, 1.0, 1.0, sc);
        BLAUNCH(k_b_xpay, grid, block, 0, ctx->stream, g, b, p_to_T1, vT2, ctx->U, 1.0, sc, part_a);
        hipLaunchKernelGGL(k_b_alpha, dim3(1), dim3(kRedBlock), 0, ctx->stream, part_a, nb, b.k, nrhs, sc);
        BLAUNCH(k_b_clovinv, grid, block, 0, ctx->stream, g, b, T1_to_T2, ctx->U, -1.0, 1.0, sc);
        BLAUNCH(k_b_hop4, grid, block, 0, ctx->stream, g, b, vT1, vT2, vP, vX, vR, ctx->U, sc, part_b);
        hipLaunchKernelGGL(k_b_beta, dim3(1), dim3(kRedBlock), 0, ctx->stream, part_b, nb, b.k, nrhs, sc);
        hipLaunchKernelGGL(k_b_update_p, dim3(nblocks(n * nrhs, 256)), dim3(256), 0, ctx->stream, g, b, vR, vP, sc);
        LAUNCHCHK(ctx);
        return 0;
    };
    std::vector<uint64_t> key;
    key_add(key, 5);   // batched CG iteration
    key_geom(key, g);
    key_add(key, nrhs);
    for (int r = 0; r < nrhs; r++) {
        for (const void *ptr : {(const void *)P[r], (const void *)T1[r], (const void *)T2[r], (const void *)R[r],
                                (const void *)x_[r], (const void *)b.clo[r], (const void *)b.cle[r]})
            key_add(key, ptr);
        key_add(key, b.a[r]);
    }
    for (const void *ptr : {(const void *)part_a, (const void *)part_b, (const void *)sc, (const void *)ctx->U})
        key_add(key, ptr);
    key_add(key, b.clov[0]);
    for (;;) {
        if ((rc = graph_run(ctx, key, chunk, iteration))) return rc;
        HIPCHK(ctx, hipMemcpyAsync(ctx->red_host, sc, sizeof(double) * 8 * kMaxRhs, hipMemcpyDeviceToHost,
                                   ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        bool all = true;
        for (int r = 0; r < nrhs; r++) {
            h[8 * r + B_DONE] = ctx->red_host[8 * r + B_DONE];
            h[8 * r + B_ITER] = ctx->red_host[8 * r + B_ITER];
            all = all && h[8 * r + B_DONE] != 0;
        }
        if (all) break;
    }
    // FP64 true residuals, one rhs at a time
    double2 *Kx = (double2 *)ws_alloc(ctx, vb, 8), *te = (double2 *)ws_alloc(ctx, vb, 6),
            *to = (double2 *)ws_alloc(ctx, vb, 7);
    if (!Kx || !te || !to) return set_err(ctx, PFMP_ERR_OOM, "batch workspace");
    int worst_rc = 0;
    for (int r = 0; r < nrhs; r++) {
        if ((rc = op_apply_K(ctx, ops[r], (const double2 *)x_[r], Kx, te, to, nullptr))) return rc;
        double one[2] = {1, 0}, mone[2] = {-1, 0};
        HIPCHK(ctx, hipMemcpyAsync(te, b_[r], vb, hipMemcpyDeviceToDevice, ctx->stream));
        if ((rc = pfmp_axpby(ctx, mone, Kx, one, te))) return rc;
        double rr;
        if ((rc = launch_norm2(ctx, te, n, ctx->red))) return rc;
        if ((rc = red_finish(ctx, ctx->red, ctx->nblk_red, 1, &rr))) return rc;
        double res = bb[r] > 0 ? std::sqrt(rr / bb[r]) : 0;
        if (st) {
            st[r].iters = (int)h[8 * r + B_ITER];
            st[r].reliable_updates = 0;
            st[r].true_res = res;
            st[r].kmults = st[r].iters + 1;
        }
        if (h[8 * r + B_DONE] == 2 && !(res <= prm->tol)) worst_rc = PFMP_ERR_NOCONV;
    }
    auto t1 = std::chrono::steady_clock::now();
    if (st)
        for (int r = 0; r < nrhs; r++) st[r].seconds = std::chrono::duration<double>(t1 - t0).count();
    if (worst_rc) return set_err(ctx, worst_rc, "cg_solve_batch: maxiter reached");
    return 0;
}
