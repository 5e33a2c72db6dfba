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
template <typename C, typename R, int CLOV, int LM>
__global__ __launch_bounds__(kBlock) void k_poly_last(Geom g, const C *__restrict__ t, const C *__restrict__ T,
                                                      const C *__restrict__ U, const R *__restrict__ cl, R a,
                                                      const C *__restrict__ src, C z, C *__restrict__ dst)
{
    const int tt = xcd_site(2 * g.Vh);
    if (tt < 0) return;
    const int i = tile_site(g, tt >> 1), hb = tt & 1;
    C acc[6], tv[6], at[6];
    hop_pair<LM, C>(g, 0, i, hb, T, U, (R)1, acc);
    load_block(t, g.Vh, i, hb, (R)-1, tv);
    if (CLOV) clover_block<R, C>(cl, g.Vh, i, hb, tv, at);
    const long Vh = g.Vh;
#pragma unroll
    for (int k = 0; k < 6; k++) {
        C base = CLOV ? at[k] : tv[k];
        C kv = mk<C>(base.x + a * acc[k].x, base.y + a * acc[k].y);
        if (hb) kv = mk<C>(-kv.x, -kv.y);
        const long e = (long)(6 * hb + k) * Vh + i;
        dst[e] = csub(kv, cmul(z, src[e]));
    }
}

template <typename C>
__global__ void k_cscale(long n, C a, const C *__restrict__ x, C *__restrict__ y)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) y[t] = cmul(a, x[t]);
}

// FP64 operator stages on the FP64 links and clover, FP32 ones on their FP32 copies
struct Stages64 {
    using C = double2;
    using R = double;
    static const C *links(pfmp_ctx *ctx) { return ctx->U; }
    static const R *clov(const OpSlot &s, int p) { return s.clov[p]; }
    static int M(pfmp_ctx *ctx, int op, const C *in, C *out, C *tmp) { return op_apply_M(ctx, op, 0, in, out, tmp, nullptr); }
    static int clovinv(pfmp_ctx *ctx, const C *in, const R *cl, C *out, bool clv)
    {
        return clovinv64(ctx, 1, in, cl, out, -1.0, 1.0, clv, nullptr);
    }
};
struct Stages32 {
    using C = float2;
    using R = float;
    static const C *links(pfmp_ctx *ctx) { return ctx->Uf; }
    static const R *clov(const OpSlot &s, int p) { return s.clovf[p]; }
    static int M(pfmp_ctx *ctx, int op, const C *in, C *out, C *tmp) { return op_apply_M_f32(ctx, op, 0, in, out, tmp, nullptr); }
    static int clovinv(pfmp_ctx *ctx, const C *in, const R *cl, C *out, bool clv)
    {
        return clovinv32(ctx, 1, in, cl, out, -1.f, 1.f, clv, nullptr);
    }
};

// dst = (Khat - z) src on slot op; dst must differ from src
template <typename S>
int poly_factor_t(pfmp_ctx *ctx, int op, const typename S::C *src, typename S::C z, typename S::C *dst,
                  typename S::C *te, typename S::C *to)
{
    using C = typename S::C;
    using R = typename S::R;
    OpSlot &s = ctx->ops[op];
    const bool cl = s.csw != 0;
    const R mk2 = (R)(-s.kappa * s.kappa);
    int rc = S::M(ctx, op, src, te, to);
    if (rc) return rc;
    if ((rc = S::clovinv(ctx, te, S::clov(s, 1), to, cl))) return rc;
    dim3 grid(op_nparts(ctx->g)), block(kBlock);
    const C *U = S::links(ctx);
    const R *c0 = S::clov(s, 0);
#define LAST(CL, LM)                                                                                               \
    hipLaunchKernelGGL((k_poly_last<C, R, CL, LM>), grid, block, 0, ctx->stream, ctx->g, te, to, U, c0, mk2, src, z, \
                       dst)
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

template <typename C>
int scale_spinor_t(pfmp_ctx *ctx, C a, const C *x, C *y)
{
    long n = 12L * ctx->g.Vh;
    hipLaunchKernelGGL(k_cscale<C>, dim3(nblocks(n, 256)), dim3(256), 0, ctx->stream, n, a, x, y);
    LAUNCHCHK(ctx);
    return 0;
}

// v_0 = norm in, v_{k+1} = (Khat - z_k) v_k in precision S
template <typename S>
int apply_poly_t(pfmp_ctx *ctx, int op, int n, const double *roots, const double norm[2], const void *in, void *out,
                 void *const *chain, size_t vb)
{
    using C = typename S::C;
    using R = typename S::R;
    C *te = (C *)ws_alloc(ctx, vb, 20), *to = (C *)ws_alloc(ctx, vb, 21);
    C *pa = (C *)ws_alloc(ctx, vb, 22), *pb = (C *)ws_alloc(ctx, vb, 23);
    if (!te || !to || !pa || !pb) return set_err(ctx, PFMP_ERR_OOM, "apply_poly workspace");
    C *cur = n == 0 ? (C *)out : (chain ? (C *)chain[0] : pa);
    int rc = scale_spinor_t<C>(ctx, mk<C>((R)norm[0], (R)norm[1]), (const C *)in, cur);
    if (rc) return rc;
    for (int k = 0; k < n; k++) {
        C *dst;
        if (k == n - 1) dst = (C *)out;
        else if (chain) dst = (C *)chain[k + 1];
        else dst = cur == pa ? pb : pa;
        if (dst == cur) return set_err(ctx, PFMP_ERR_ARG, "apply_poly: out aliases a chain buffer");
        if ((rc = poly_factor_t<S>(ctx, op, cur, mk<C>((R)roots[2 * k], (R)roots[2 * k + 1]), dst, te, to))) return rc;
        cur = dst;
    }
    return 0;
}

}  // namespace

int poly_factor(pfmp_ctx *ctx, int op, const double2 *src, double2 z, double2 *dst, double2 *te, double2 *to)
{
    return poly_factor_t<Stages64>(ctx, op, src, z, dst, te, to);
}

int scale_spinor(pfmp_ctx *ctx, double2 a, const double2 *x, double2 *y) { return scale_spinor_t<double2>(ctx, a, x, y); }

extern "C" int pfmp_apply_poly(pfmp_ctx *ctx, int op, int n, const double *roots, const double norm[2],
                               const void *in, void *out, void *const *chain, int prec)
{
    if (!ctx) return PFMP_ERR_ARG;
    if (op < 0 || op >= PFMP_MAX_OPS || !ctx->have_gauge || !ctx->ops[op].valid)
        return set_err(ctx, PFMP_ERR_STATE, "apply_poly: operator not configured");
    if (int rc0 = op_ready(ctx, op)) return rc0;
    if (n < 0 || (n > 0 && !roots) || !norm || !in || !out)
        return set_err(ctx, PFMP_ERR_ARG, "apply_poly: bad arguments");
    if (prec != PFMP_F64 && prec != PFMP_F32) return set_err(ctx, PFMP_ERR_ARG, "apply_poly: FP64 or FP32 only");
    if (chain)
        for (int k = 0; k < n; k++)
            if (!chain[k]) return set_err(ctx, PFMP_ERR_ARG, "apply_poly: null chain buffer");
    size_t vb = sizeof(double) * spinor_reals(ctx->g);
    if (prec == PFMP_F64) return apply_poly_t<Stages64>(ctx, op, n, roots, norm, in, out, chain, vb);
    if (int rc = gauge_f32_ready(ctx)) return rc;
    return apply_poly_t<Stages32>(ctx, op, n, roots, norm, in, out, chain, vb / 2);
}
