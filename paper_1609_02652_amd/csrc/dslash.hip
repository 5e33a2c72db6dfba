// dslash.hip -- even-odd Wilson-clover operator kernels for gfx950 (hopping
// term building blocks in hop.h).
//
// Stages (paper Sec. 2.1 operator, even-odd Schur form):
//   hop_clovinv : out_o = [g5] A_oo^-1 D_oe [g5] in_e      (also plain D for tests)
//   hop_xpay    : out_e = [g5] (A_ee [g5] x_e + a D_eo t_o), optional |out|^2 partials
// Mhat = both stages (a = -kappa^2); Mhat^dag = the same with g5 on input and output.
#include <mutex>

#include "hop.h"

namespace {

// out = [g5] A^-1 D in [g5], output parity pout (CLOV = 0: no clover); In / Out are
// spinor pointers of the register type C or FP16 storage (HalfField).  Two lanes per
// site, lane hb writing chiral block hb.
template <typename C, typename R, int CLOV, int LM, typename In, typename Out, typename UL, typename CL>
__global__ __launch_bounds__(kBlock) void k_hop_clovinv(Geom g, int pout, const In in, UL U, CL cl, Out out, R gin,
                                                        R gout, const double *__restrict__ stop)
{
    if (stop && stop[0] != 0) return;
    const int tt = xcd_site(2 * g.Vh);
    if (tt < 0) return;
    const int i = tile_site(g, tt >> 1), hb = tt & 1;
    C blk[6];
    hop_pair<LM, C>(g, pout, i, hb, in, U, gin, blk);
    if (CLOV) {
        C t[6];
        clover_block<R, C>(cl, g.Vh, i, hb, blk, t);
        store_block_st<(LM >> 1) & 1>(out, g.Vh, i, hb, gout, t);
    } else {
        store_block_st<(LM >> 1) & 1>(out, g.Vh, i, hb, gout, blk);
    }
}

// out = [g5] (A [g5] x + a D t), output parity pout; NORM: |out|^2 block partials
template <typename C, typename R, int CLOV, int NORM, int LM, typename X, typename T, typename Out, typename UL,
          typename CL>
__global__ __launch_bounds__(kBlock) void k_hop_xpay(Geom g, int pout, const X x, const T t, UL U, CL cl, R a,
                                                     Out out, R gs, double *partials, const double *__restrict__ stop)
{
    if (stop && stop[0] != 0) return;
    const int tt = xcd_site(2 * g.Vh);
    double nrm = 0;
    if (tt >= 0) {
        const int i = tile_site(g, tt >> 1), hb = tt & 1;
        C acc[6], xv[6], ax[6];
        hop_pair<LM, C>(g, pout, i, hb, t, U, (R)1, acc);
        load_block_st<(LM >> 1) & 1>(x, g.Vh, i, hb, gs, xv);
        if (CLOV) clover_block<R, C>(cl, g.Vh, i, hb, xv, ax);
#pragma unroll
        for (int k = 0; k < 6; k++) {
            C base = CLOV ? ax[k] : xv[k];
            acc[k] = mk<C>(fmadd(a, acc[k].x, base.x), fmadd(a, acc[k].y, base.y));
            if (NORM) cnorm_acc(nrm, acc[k]);
        }
        store_block_st<(LM >> 1) & 1>(out, g.Vh, i, hb, gs, acc);
    }
    if (NORM) {
        const double v[1] = {nrm};
        op_partials_store<kBlock, 1>(v, partials);
    }
}

}  // namespace

template <typename C, typename R, typename In, typename Out, typename UL, typename CL>
int launch_clovinv(pfmp_ctx *ctx, int pout, In in, UL U, CL cl, Out out, R gin, R gout, bool clov,
                   const double *stop)
{
    dim3 grid(op_nparts(ctx->g)), block(kBlock);
#define CLOVINV(CV, LM)                                                                                           \
    hipLaunchKernelGGL((k_hop_clovinv<C, R, CV, LM, In, Out, UL, CL>), grid, block, 0, ctx->stream, ctx->g, pout, in, \
                       U, cl, out, gin, gout, stop)
#define CLOVINV1(LM) CLOVINV(1, LM)
#define CLOVINV0(LM) CLOVINV(0, LM)
    const int lm = link_mode(ctx->g);
    if (clov) { PFMP_LM_SWITCH(lm, CLOVINV1) }
    else { PFMP_LM_SWITCH(lm, CLOVINV0) }
#undef CLOVINV1
#undef CLOVINV0
#undef CLOVINV
    LAUNCHCHK(ctx);
    return 0;
}

template <typename C, typename R, typename X, typename T, typename Out, typename UL, typename CL>
int launch_xpay(pfmp_ctx *ctx, int pout, X x, T t, UL U, CL cl, R a, Out out, R gs, bool clov, double *partials,
                const double *stop)
{
    dim3 grid(op_nparts(ctx->g)), block(kBlock);
#define XPAY(CV, NM, LM)                                                                                           \
    hipLaunchKernelGGL((k_hop_xpay<C, R, CV, NM, LM, X, T, Out, UL, CL>), grid, block, 0, ctx->stream, ctx->g, pout, \
                       x, t, U, cl, a, out, gs, partials, stop)
#define XPAY11(LM) XPAY(1, 1, LM)
#define XPAY10(LM) XPAY(1, 0, LM)
#define XPAY01(LM) XPAY(0, 1, LM)
#define XPAY00(LM) XPAY(0, 0, LM)
    const int lm = link_mode(ctx->g);
    if (clov && partials) { PFMP_LM_SWITCH(lm, XPAY11) }
    else if (clov) { PFMP_LM_SWITCH(lm, XPAY10) }
    else if (partials) { PFMP_LM_SWITCH(lm, XPAY01) }
    else { PFMP_LM_SWITCH(lm, XPAY00) }
#undef XPAY11
#undef XPAY10
#undef XPAY01
#undef XPAY00
#undef XPAY
    LAUNCHCHK(ctx);
    return 0;
}

template int launch_clovinv<double2, double, const double2 *, double2 *, const double2 *, const double *>(
    pfmp_ctx *, int, const double2 *, const double2 *, const double *, double2 *, double, double, bool,
    const double *);
template int launch_clovinv<float2, float, const float2 *, float2 *, const float2 *, const float *>(
    pfmp_ctx *, int, const float2 *, const float2 *, const float *, float2 *, float, float, bool, const double *);
template int launch_clovinv<float2, float, HalfField, HalfField, HalfLinks, HalfClover>(pfmp_ctx *, int, HalfField,
                                                                                       HalfLinks, HalfClover,
                                                                                       HalfField, float, float, bool,
                                                                                       const double *);
template int launch_xpay<double2, double, const double2 *, const double2 *, double2 *, const double2 *,
                         const double *>(pfmp_ctx *, int, const double2 *, const double2 *, const double2 *,
                                         const double *, double, double2 *, double, bool, double *, const double *);
template int launch_xpay<float2, float, const float2 *, const float2 *, float2 *, const float2 *, const float *>(
    pfmp_ctx *, int, const float2 *, const float2 *, const float2 *, const float *, float, float2 *, float, bool,
    double *, const double *);
template int launch_xpay<float2, float, HalfField, HalfField, HalfField, HalfLinks, HalfClover>(
    pfmp_ctx *, int, HalfField, HalfField, HalfLinks, HalfClover, float, HalfField, float, bool, double *,
    const double *);
template int launch_clovinv<float2, float, HalfField, HalfField, const float2 *, const float *>(
    pfmp_ctx *, int, HalfField, const float2 *, const float *, HalfField, float, float, bool, const double *);
template int launch_xpay<float2, float, HalfField, HalfField, HalfField, const float2 *, const float *>(
    pfmp_ctx *, int, HalfField, HalfField, const float2 *, const float *, float, HalfField, float, bool, double *,
    const double *);

namespace {

// clover (or inverse) on one parity
template <typename C, typename R>
__global__ __launch_bounds__(kBlock) void k_clover(Geom g, const C *__restrict__ in, const R *__restrict__ cl,
                                                   C *__restrict__ out)
{
    int i = xcd_site(g.Vh);
    if (i < 0) return;
    C v[12], w[12];
    load_spinor(in, g.Vh, i, (R)1, v);
    clover_apply<R, C>(cl, g.Vh, i, v, w);
    store_spinor(out, g.Vh, i, (R)1, w);
}

// FP32 spinor (one parity) into FP16 storage (per-site scale) and back
__global__ __launch_bounds__(kBlock) void k_to_half(int Vh, const float2 *__restrict__ in, HalfField out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Vh) return;
    float2 v[12];
    load_spinor(in, Vh, i, 1.f, v);
    store_spinor(out, Vh, i, 1.f, v);
}

__global__ __launch_bounds__(kBlock) void k_from_half(int Vh, HalfField in, float2 *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Vh) return;
    float2 v[12];
    load_spinor(in, Vh, i, 1.f, v);
    store_spinor(out, Vh, i, 1.f, v);
}

}  // namespace

// ------------------------------------------------------------------ internal API

static bool op_has_clover(const OpSlot &s) { return s.csw != 0; }

int op_apply_M(pfmp_ctx *ctx, int op, int dagger, const double2 *in, double2 *out, double2 *tmp_odd,
               double *norm_partials)
{
    OpSlot &s = ctx->ops[op];
    double gs = dagger ? -1.0 : 1.0;
    bool cl = op_has_clover(s);
    int rc = launch_clovinv<double2, double, const double2 *, double2 *, const double2 *, const double *>(ctx, 1, in, ctx->U, s.clov[1], tmp_odd, gs, 1.0, cl, nullptr);
    if (rc) return rc;
    return launch_xpay<double2, double, const double2 *, const double2 *, double2 *, const double2 *, const double *>(ctx, 0, in, tmp_odd, ctx->U, s.clov[0], -s.kappa * s.kappa, out, gs, cl,
                                        norm_partials, nullptr);
}

int op_apply_K(pfmp_ctx *ctx, int op, const double2 *in, double2 *out, double2 *tmp_even, double2 *tmp_odd,
               double *norm_partials)
{
    int rc = op_apply_M(ctx, op, 0, in, tmp_even, tmp_odd, norm_partials);
    if (rc) return rc;
    return op_apply_M(ctx, op, 1, tmp_even, out, tmp_odd, nullptr);
}

int op_apply_M_f32(pfmp_ctx *ctx, int op, int dagger, const float2 *in, float2 *out, float2 *tmp_odd,
                   double *norm_partials)
{
    OpSlot &s = ctx->ops[op];
    float gs = dagger ? -1.f : 1.f;
    bool cl = op_has_clover(s);
    int rc = launch_clovinv<float2, float, const float2 *, float2 *, const float2 *, const float *>(ctx, 1, in, ctx->Uf, s.clovf[1], tmp_odd, gs, 1.f, cl, nullptr);
    if (rc) return rc;
    return launch_xpay<float2, float, const float2 *, const float2 *, float2 *, const float2 *, const float *>(ctx, 0, in, tmp_odd, ctx->Uf, s.clovf[0], (float)(-s.kappa * s.kappa), out,
                                      gs, cl, norm_partials, nullptr);
}

int op_apply_K_f32(pfmp_ctx *ctx, int op, const float2 *in, float2 *out, float2 *tmp_even, float2 *tmp_odd,
                   double *norm_partials)
{
    int rc = op_apply_M_f32(ctx, op, 0, in, tmp_even, tmp_odd, norm_partials);
    if (rc) return rc;
    return op_apply_M_f32(ctx, op, 1, tmp_even, out, tmp_odd, nullptr);
}

// Mhat (dagger) or Khat (K = 1) with FP16 spinor storage: in and out are FP32 spinors; the
// input is rounded into FP16 storage, each stage stores its result in FP16 storage (FP32
// arithmetic), as the FP16-storage inner solver does, and the result is widened to FP32.
// Links and clover: the FP16 copies, or the FP32 ones when half links are off.
template <typename UL, typename CL>
static int apply_half(pfmp_ctx *ctx, int op, int dagger, int K, const float2 *in, float2 *out, UL U, CL c0, CL c1)
{
    const Geom &g = ctx->g;
    const OpSlot &s = ctx->ops[op];
    const size_t hb = 4L * 12 * g.Vh + 4L * g.Vh;
    void *b0 = ws_alloc(ctx, hb, 40), *b1 = ws_alloc(ctx, hb, 41), *b2 = ws_alloc(ctx, hb, 42);
    if (!b0 || !b1 || !b2) return set_err(ctx, PFMP_ERR_OOM, "workspace");
    auto half = [&](void *p) { return HalfField{(H3 *)p, (float *)((char *)p + 4L * 12 * g.Vh)}; };
    HalfField hin = half(b0), htmp = half(b1), hout = half(b2);
    const bool cl = op_has_clover(s);
    const float mk2 = (float)(-s.kappa * s.kappa);
    hipLaunchKernelGGL(k_to_half, dim3(nblocks(g.Vh, kBlock)), dim3(kBlock), 0, ctx->stream, g.Vh, in, hin);
    LAUNCHCHK(ctx);
    int rc;
    for (int pass = 0; pass < (K ? 2 : 1); pass++) {
        const float gs = (K ? pass == 1 : dagger != 0) ? -1.f : 1.f;
        HalfField src = pass == 0 ? hin : hout, dst = pass == 0 ? hout : hin;
        if ((rc = launch_clovinv<float2, float, HalfField, HalfField, UL, CL>(ctx, 1, src, U, c1, htmp, gs, 1.f, cl,
                                                                               nullptr)))
            return rc;
        if ((rc = launch_xpay<float2, float, HalfField, HalfField, HalfField, UL, CL>(ctx, 0, src, htmp, U, c0, mk2, dst,
                                                                                       gs, cl, nullptr, nullptr)))
            return rc;
    }
    hipLaunchKernelGGL(k_from_half, dim3(nblocks(g.Vh, kBlock)), dim3(kBlock), 0, ctx->stream, g.Vh,
                       K ? hin : hout, out);
    LAUNCHCHK(ctx);
    return 0;
}

static int apply_f16(pfmp_ctx *ctx, int op, int dagger, int K, const void *in, void *out)
{
    const OpSlot &s = ctx->ops[op];
    if (ctx->half_links)
        return apply_half<HalfLinks, HalfClover>(ctx, op, dagger, K, (const float2 *)in, (float2 *)out,
                                                 HalfLinks{(const __half2 *)ctx->Uh},
                                                 HalfClover{(const H3 *)s.clovh[0]},
                                                 HalfClover{(const H3 *)s.clovh[1]});
    return apply_half<const float2 *, const float *>(ctx, op, dagger, K, (const float2 *)in, (float2 *)out, ctx->Uf,
                                                     s.clovf[0], s.clovf[1]);
}

// ------------------------------------------------------------------ C-ABI

static int check_op(pfmp_ctx *ctx, int op)
{
    if (!ctx) return PFMP_ERR_ARG;
    if (op < 0 || op >= PFMP_MAX_OPS) return set_err(ctx, PFMP_ERR_ARG, "operator slot out of range");
    if (!ctx->have_gauge) return set_err(ctx, PFMP_ERR_STATE, "no gauge field set");
    if (!ctx->ops[op].valid) return set_err(ctx, PFMP_ERR_STATE, "operator slot not configured");
    int rc = op_ready(ctx, op);
    return rc ? rc : gauge_f32_ready(ctx);
}

extern "C" int pfmp_apply_hop(pfmp_ctx *ctx, int out_parity, int dagger, const void *in, void *out)
{
    if (!ctx || !in || !out || (out_parity != 0 && out_parity != 1)) return ctx ? set_err(ctx, PFMP_ERR_ARG, "apply_hop: bad argument") : PFMP_ERR_ARG;
    if (!ctx->have_gauge) return set_err(ctx, PFMP_ERR_STATE, "no gauge field set");
    double gs = dagger ? -1.0 : 1.0;
    return launch_clovinv<double2, double, const double2 *, double2 *, const double2 *, const double *>(ctx, out_parity, (const double2 *)in, ctx->U, nullptr, (double2 *)out, gs,
                                           gs, false, nullptr);
}

extern "C" int pfmp_apply_clover(pfmp_ctx *ctx, int op, int parity, int inverse, const void *in, void *out)
{
    int rc = check_op(ctx, op);
    if (rc) return rc;
    if (!in || !out || (parity != 0 && parity != 1)) return set_err(ctx, PFMP_ERR_ARG, "apply_clover: bad argument");
    if (inverse != (parity == 1)) return set_err(ctx, PFMP_ERR_ARG, "apply_clover: the context holds A_ee and A_oo^-1");
    OpSlot &s = ctx->ops[op];
    if (!op_has_clover(s)) {
        HIPCHK(ctx, hipMemcpyAsync(out, in, sizeof(double) * spinor_reals(ctx->g), hipMemcpyDeviceToDevice, ctx->stream));
        return 0;
    }
    hipLaunchKernelGGL((k_clover<double2, double>), dim3(nblocks_site(ctx->g.Vh)), dim3(kBlock), 0, ctx->stream,
                       ctx->g, (const double2 *)in, s.clov[parity], (double2 *)out);
    LAUNCHCHK(ctx);
    return 0;
}

extern "C" int pfmp_apply_M(pfmp_ctx *ctx, int op, int dagger, const void *in, void *out, int prec)
{
    int rc = check_op(ctx, op);
    if (rc) return rc;
    if (!in || !out) return set_err(ctx, PFMP_ERR_ARG, "apply_M: null buffer");
    if (prec == PFMP_F64) {
        double2 *tmp = (double2 *)ws_alloc(ctx, sizeof(double) * spinor_reals(ctx->g), 0);
        if (!tmp) return set_err(ctx, PFMP_ERR_OOM, "workspace");
        return op_apply_M(ctx, op, dagger, (const double2 *)in, (double2 *)out, tmp, nullptr);
    }
    if (prec == PFMP_F32) {
        float2 *tmp = (float2 *)ws_alloc(ctx, sizeof(float) * spinor_reals(ctx->g), 1);
        if (!tmp) return set_err(ctx, PFMP_ERR_OOM, "workspace");
        return op_apply_M_f32(ctx, op, dagger, (const float2 *)in, (float2 *)out, tmp, nullptr);
    }
    if (prec == PFMP_F16) return apply_f16(ctx, op, dagger, 0, in, out);
    return set_err(ctx, PFMP_ERR_ARG, "apply_M: unsupported precision");
}

// ------------------------------------------------------------------ allocation-free Khat
//
// Scratch of pfmp_apply_MdagM_noalloc: the even and odd intermediates of Khat in one
// statically allocated device array (each GPU holds its own copy from module load until
// the process ends).  Host code never passes the array's name to a kernel: its device
// address on each GPU is looked up once, at context creation with that GPU current
// (noalloc_scratch_init), and kept per device.
constexpr size_t kScratchBytes = 128ull << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_dev[kMaxDevices] = {};
}  // namespace

int noalloc_scratch_init(pfmp_ctx *ctx)
{
    int dev = 0;
    HIPCHK(ctx, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_err(ctx, PFMP_ERR_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        HIPCHK(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_err(ctx, PFMP_ERR_HIP, "scratch: no device address");
        scratch_dev[dev] = p;
    }
    ctx->scratch = scratch_dev[dev];
    return 0;
}

extern "C" int pfmp_apply_MdagM_noalloc(pfmp_ctx *ctx, int op, const void *in, void *out, int prec)
{
    if (!ctx) return PFMP_ERR_ARG;
    if (op < 0 || op >= PFMP_MAX_OPS) return set_err(ctx, PFMP_ERR_ARG, "operator slot out of range");
    if (!in || !out) return set_err(ctx, PFMP_ERR_ARG, "apply_MdagM_noalloc: null buffer");
    if (prec != PFMP_F64 && prec != PFMP_F32)
        return set_err(ctx, PFMP_ERR_ARG, "apply_MdagM_noalloc: FP64 or FP32 fields only");
    const size_t field = (prec == PFMP_F64 ? sizeof(double) : sizeof(float)) * spinor_reals(ctx->g);
    if (2 * field > kScratchBytes)
        return set_err(ctx, PFMP_ERR_ARG, "apply_MdagM_noalloc: lattice too large for the 128 MiB scratch (two "
                                          "spinor fields of one parity)");
    if (!ctx->scratch) return set_err(ctx, PFMP_ERR_STATE, "apply_MdagM_noalloc: scratch not set up");
    // a stale clover slot is rebuilt in place (its buffers exist from pfmp_set_operator)
    if (!ctx->have_gauge) return set_err(ctx, PFMP_ERR_STATE, "no gauge field set");
    if (!ctx->ops[op].valid) return set_err(ctx, PFMP_ERR_STATE, "operator slot not configured");
    if (ctx->ops[op].stale && !(ctx->Fhat && ctx->ops[op].ldpart))
        return set_err(ctx, PFMP_ERR_STATE, "apply_MdagM_noalloc: clover fields not allocated");
    int rc = op_ready(ctx, op);
    if (!rc) rc = gauge_f32_ready(ctx);
    if (rc) return rc;
    char *te = (char *)ctx->scratch, *to = te + field;
    if (prec == PFMP_F64)
        return op_apply_K(ctx, op, (const double2 *)in, (double2 *)out, (double2 *)te, (double2 *)to, nullptr);
    return op_apply_K_f32(ctx, op, (const float2 *)in, (float2 *)out, (float2 *)te, (float2 *)to, nullptr);
}

extern "C" int pfmp_apply_MdagM(pfmp_ctx *ctx, int op, const void *in, void *out, int prec)
{
    int rc = check_op(ctx, op);
    if (rc) return rc;
    if (!in || !out) return set_err(ctx, PFMP_ERR_ARG, "apply_MdagM: null buffer");
    if (prec == PFMP_F64) {
        double2 *te = (double2 *)ws_alloc(ctx, sizeof(double) * spinor_reals(ctx->g), 0);
        double2 *to = (double2 *)ws_alloc(ctx, sizeof(double) * spinor_reals(ctx->g), 2);
        if (!te || !to) return set_err(ctx, PFMP_ERR_OOM, "workspace");
        return op_apply_K(ctx, op, (const double2 *)in, (double2 *)out, te, to, nullptr);
    }
    if (prec == PFMP_F32) {
        float2 *te = (float2 *)ws_alloc(ctx, sizeof(float) * spinor_reals(ctx->g), 1);
        float2 *to = (float2 *)ws_alloc(ctx, sizeof(float) * spinor_reals(ctx->g), 3);
        if (!te || !to) return set_err(ctx, PFMP_ERR_OOM, "workspace");
        return op_apply_K_f32(ctx, op, (const float2 *)in, (float2 *)out, te, to, nullptr);
    }
    if (prec == PFMP_F16) return apply_f16(ctx, op, 0, 1, in, out);
    return set_err(ctx, PFMP_ERR_ARG, "apply_MdagM: unsupported precision");
}
