// poly.hip -- product-form polynomial filter P(Khat) = a_n prod_k (Khat - z_k)
// (paper App. A) with the intermediate vectors the polynomial force needs
// (App. C, eq. force_poly).
//
// v_0 = norm * in, v_{k+1} = Khat v_k - z_k v_k; chain[k] = v_k; out = v_n.
// Each factor is one Khat multiplication: 3 hopping launches plus a fused last
// launch that forms Khat v and subtracts z v in its epilogue.
#include "hop.h"

namespace {

// dst = g5 (A_ee g5 t - kappa^2 D_eo T') - z src, with t = Mhat src, T' = A_oo^-1 D_oe g5 t
template <int CLOV, int LM>
__global__ __launch_bounds__(kBlock) void k_poly_last(Geom g, const double2 *__restrict__ t,
                                                      const double2 *__restrict__ T, const double2 *__restrict__ U,
                                                      const double *__restrict__ cl, double a,
                                                      const double2 *__restrict__ src, double2 z,
                                                      double2 *__restrict__ dst)
{
    const int tt = xcd_site(2 * g.Vh);
    if (tt < 0) return;
    const int i = tile_site(g, tt >> 1), hb = tt & 1;
    double2 acc[6], tv[6], at[6];
    hop_pair<LM, double2>(g, 0, i, hb, T, U, 1.0, acc);
    load_block(t, g.Vh, i, hb, -1.0, tv);
    if (CLOV) clover_block<double, double2>(cl, g.Vh, i, hb, tv, at);
    const long Vh = g.Vh;
#pragma unroll
    for (int k = 0; k < 6; k++) {
        double2 base = CLOV ? at[k] : tv[k];
        double2 kv = make_double2(base.x + a * acc[k].x, base.y + a * acc[k].y);
        if (hb) kv = cneg(kv);
        const long e = (long)(6 * hb + k) * Vh + i;
        dst[e] = csub(kv, cmul(z, src[e]));
    }
}

__global__ void k_cscale(long n, double2 a, const double2 *__restrict__ x, double2 *__restrict__ y)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) y[t] = cmul(a, x[t]);
}

}  // namespace

// dst = (Khat - z) src on slot op (FP64); dst must differ from src
int poly_factor(pfmp_ctx *ctx, int op, const double2 *src, double2 z, double2 *dst, double2 *te, double2 *to)
{
    OpSlot &s = ctx->ops[op];
    const bool cl = s.csw != 0;
    const double mk2 = -s.kappa * s.kappa;
    int rc = op_apply_M(ctx, op, 0, src, te, to, nullptr);
    if (rc) return rc;
    if ((rc = clovinv64(ctx, 1, te, s.clov[1], to, -1.0, 1.0, cl, nullptr))) return rc;
    dim3 grid(op_nparts(ctx->g)), block(kBlock);
#define LAST(CL, LM)                                                                                          \
    hipLaunchKernelGGL((k_poly_last<CL, LM>), grid, block, 0, ctx->stream, ctx->g, te, to, ctx->U, s.clov[0], mk2, \
                       src, z, dst)
#define LAST1(LM) LAST(1, LM)
#define LAST0(LM) LAST(0, LM)
    if (cl) { PFMP_LM_SWITCH(link_mode(ctx->g), LAST1) }
    else { PFMP_LM_SWITCH(link_mode(ctx->g), LAST0) }
#undef LAST1
#undef LAST0
#undef LAST
    LAUNCHCHK(ctx);
    return 0;
}

int scale_spinor(pfmp_ctx *ctx, double2 a, const double2 *x, double2 *y)
{
    long n = 12L * ctx->g.Vh;
    hipLaunchKernelGGL(k_cscale, dim3(nblocks(n, 256)), dim3(256), 0, ctx->stream, n, a, x, y);
    LAUNCHCHK(ctx);
    return 0;
}

extern "C" int pfmp_apply_poly(pfmp_ctx *ctx, int op, int n, const double *roots, const double norm[2],
                               const void *in, void *out, void *const *chain, int prec)
{
    if (!ctx) return PFMP_ERR_ARG;
    if (op < 0 || op >= PFMP_MAX_OPS || !ctx->have_gauge || !ctx->ops[op].valid)
        return set_err(ctx, PFMP_ERR_STATE, "apply_poly: operator not configured");
    if (int rc0 = op_ready(ctx, op)) return rc0;
    if (n < 0 || (n > 0 && !roots) || !norm || !in || !out)
        return set_err(ctx, PFMP_ERR_ARG, "apply_poly: bad arguments");
    if (prec != PFMP_F64) return set_err(ctx, PFMP_ERR_ARG, "apply_poly: FP64 only");
    if (chain)
        for (int k = 0; k < n; k++)
            if (!chain[k]) return set_err(ctx, PFMP_ERR_ARG, "apply_poly: null chain buffer");
    size_t vb = sizeof(double) * spinor_reals(ctx->g);
    double2 *te = (double2 *)ws_alloc(ctx, vb, 20), *to = (double2 *)ws_alloc(ctx, vb, 21);
    double2 *pa = (double2 *)ws_alloc(ctx, vb, 22), *pb = (double2 *)ws_alloc(ctx, vb, 23);
    if (!te || !to || !pa || !pb) return set_err(ctx, PFMP_ERR_OOM, "apply_poly workspace");
    double2 nm = make_double2(norm[0], norm[1]);
    // v_0 = norm * in
    double2 *cur = n == 0 ? (double2 *)out : (chain ? (double2 *)chain[0] : pa);
    int rc = scale_spinor(ctx, nm, (const double2 *)in, cur);
    if (rc) return rc;
    for (int k = 0; k < n; k++) {
        double2 *dst;
        if (k == n - 1) dst = (double2 *)out;
        else if (chain) dst = (double2 *)chain[k + 1];
        else dst = cur == pa ? pb : pa;
        if (dst == cur) return set_err(ctx, PFMP_ERR_ARG, "apply_poly: out aliases a chain buffer");
        if ((rc = poly_factor(ctx, op, cur, make_double2(roots[2 * k], roots[2 * k + 1]), dst, te, to))) return rc;
        cur = dst;
    }
    return 0;
}
