// context.hip -- context lifetime, layout conversion and index tables of libpfmp.
#include <cstring>
#include <vector>

#include <hip/hip_fp16.h>

#include "internal.h"

// Scratch buffers of the context, one per slot:
//   0-3 operator temporaries, 4-10 CG, 11-13 multi-shift, 14 link accumulator,
//   15 reduction partials, 16-19 forces, 20-23 polynomial, 24-26 trajectory,
//   27-31 mixed precision, 32-38 learned preconditioner, 40-42 FP16-storage operator.
constexpr int kWsSlots = 48;
struct SolverWS {
    void *buf[kWsSlots] = {};
    size_t bytes[kWsSlots] = {};
};

int set_err(pfmp_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

// Per-context scratch buffers keyed by slot, grown on demand and owned by the context.
void *ws_alloc(pfmp_ctx *ctx, size_t bytes, int slot)
{
    SolverWS *w = ctx->ws;
    if (slot < 0 || slot >= kWsSlots) return nullptr;
    if (w->bytes[slot] >= bytes) return w->buf[slot];
    if (w->buf[slot]) {
        hipStreamSynchronize(ctx->stream);
        hipFree(w->buf[slot]);
        w->buf[slot] = nullptr;
        w->bytes[slot] = 0;
    }
    if (hipMalloc(&w->buf[slot], bytes) != hipSuccess) {
        w->buf[slot] = nullptr;
        return nullptr;
    }
    w->bytes[slot] = bytes;
    return w->buf[slot];
}

#ifndef PFMP_UNROLL
#define PFMP_UNROLL 4
#endif

namespace {
// the executable graph of `copies` back-to-back issues of the launches (captured on first use)
int graph_get(pfmp_ctx *ctx, const std::vector<uint64_t> &key0, int copies, const std::function<int()> &issue,
              hipGraphExec_t *out)
{
    std::vector<uint64_t> key = key0;
    key.push_back(0x5eed0000u + (uint64_t)copies);
    hipGraphExec_t exec = nullptr;
    for (size_t k = 0; k < ctx->graphs.size(); k++)
        if (ctx->graphs[k].key == key) {
            exec = ctx->graphs[k].exec;
            break;
        }
    if (!exec) {
        if (!ctx->cap) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
        hipStream_t orig = ctx->stream;
        HIPCHK(ctx, hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
        ctx->stream = ctx->cap;
        int rc = 0;
        for (int c = 0; c < copies && !rc; c++) rc = issue();
        ctx->stream = orig;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->cap, &graph);
        if (rc || e != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            return rc ? rc : set_err(ctx, PFMP_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
        }
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) return set_err(ctx, PFMP_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        if (ctx->graphs.size() >= 64) {
            hipGraphExecDestroy(ctx->graphs.front().exec);
            ctx->graphs.erase(ctx->graphs.begin());
        }
        ctx->graphs.push_back({key, exec});
    }
    *out = exec;
    return 0;
}
}  // namespace

// reps issues of one iteration's launches: graphs of PFMP_UNROLL iterations, then single
// iterations for the rest (one graph launch per iteration would leave the GPU idle between them)
int graph_run(pfmp_ctx *ctx, const std::vector<uint64_t> &key, int reps, const std::function<int()> &issue)
{
    if (!ctx->use_graphs) {
        for (int r = 0; r < reps; r++)
            if (int rc = issue()) return rc;
        return 0;
    }
    hipGraphExec_t exec = nullptr;
    int rc;
    const int nu = PFMP_UNROLL > 1 ? reps / PFMP_UNROLL : 0;
    if (nu > 0) {
        if ((rc = graph_get(ctx, key, PFMP_UNROLL, issue, &exec))) return rc;
        for (int r = 0; r < nu; r++) HIPCHK(ctx, hipGraphLaunch(exec, ctx->stream));
    }
    const int rest = reps - nu * PFMP_UNROLL;
    if (rest > 0) {
        if ((rc = graph_get(ctx, key, 1, issue, &exec))) return rc;
        for (int r = 0; r < rest; r++) HIPCHK(ctx, hipGraphLaunch(exec, ctx->stream));
    }
    return 0;
}

extern "C" int pfmp_set_half_links(pfmp_ctx *ctx, int on)
{
    if (!ctx) return PFMP_ERR_ARG;
    ctx->half_links = on != 0;
    return 0;
}

extern "C" int pfmp_set_verbose(pfmp_ctx *ctx, int level)
{
    if (!ctx) return PFMP_ERR_ARG;
    ctx->verbose = level;
    return 0;
}

extern "C" int pfmp_set_graphs(pfmp_ctx *ctx, int on)
{
    if (!ctx) return PFMP_ERR_ARG;
    ctx->use_graphs = on != 0;
    return 0;
}

// Buffer idx of the context's pool of FP64 spinors; only the indices asked for
// are allocated (on first use).
double2 *pool_get(pfmp_ctx *ctx, int idx)
{
    if (idx < 0 || idx >= 4096) return nullptr;
    if ((int)ctx->pool.size() <= idx) ctx->pool.resize(idx + 1, nullptr);
    if (!ctx->pool[idx]) {
        double2 *p = nullptr;
        if (hipMalloc(&p, sizeof(double) * spinor_reals(ctx->g)) != hipSuccess) return nullptr;
        ctx->pool[idx] = p;
    }
    return ctx->pool[idx];
}

namespace {

// canonical gauge [V][4][3][3] complex128 -> internal [2][4][9][Vh]
__global__ void k_pack_gauge(Geom g, const double2 *__restrict__ in, double2 *__restrict__ U, int unpack)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= 2L * g.Vh) return;
    int p = (int)(t / g.Vh), i = (int)(t % g.Vh);
    int c[4];
    eo_coords(g, p, i, c);
    long lex = c[0] + (long)g.L[0] * (c[1] + (long)g.L[1] * (c[2] + (long)g.L[2] * c[3]));
    for (int mu = 0; mu < 4; mu++)
        for (int k = 0; k < 9; k++) {
            long ii = ((long)(p * 4 + mu) * 9 + k) * g.Vh + i;
            long cc = (lex * 4 + mu) * 9 + k;
            if (unpack) ((double2 *)in)[cc] = U[ii];
            else U[ii] = in[cc];
        }
}

// FP32 and FP16 copies of the links, each the FP64 value rounded once to nearest (the FP16
// copy is not rounded through FP32).  Element k of link l (9 Vh planes per link, k = 3 row +
// column) at site i: plane (9 l + k) Vh + i in FP64; in the FP32 and FP16 copies the row is
// one record, complex 9 l Vh + 3 row Vh + 3 i + column.
__global__ void k_gauge_f32(long Vh, long n, const double2 *__restrict__ a, float2 *__restrict__ b,
                            __half2 *__restrict__ h)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) {
        const long l = t / (9 * Vh), r = t - l * 9 * Vh, k = r / Vh, i = r - k * Vh;
        const long o = l * 9 * Vh + (k / 3) * 3 * Vh + 3 * i + k % 3;
        b[o] = make_float2((float)a[t].x, (float)a[t].y);
        h[o] = __half2{_Float16_2{static_cast<_Float16>(a[t].x), static_cast<_Float16>(a[t].y)}};
    }
}

// canonical spinor [Vh][12] complex128 <-> internal [12][Vh]
template <typename C>
__global__ void k_pack_spinor(int Vh, const double2 *__restrict__ can, C *__restrict__ f, int unpack)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= 12L * Vh) return;
    int i = (int)(t / 12), k = (int)(t % 12);
    long ii = (long)k * Vh + i;
    if (unpack) {
        C v = f[ii];
        ((double2 *)can)[t] = make_double2((double)v.x, (double)v.y);
    } else {
        double2 v = can[t];
        C w;
        w.x = v.x;
        w.y = v.y;
        f[ii] = w;
    }
}

// canonical momenta [V][4][8] <-> internal [2][4][8][Vh]
__global__ void k_pack_mom(Geom g, const double *__restrict__ can, double *__restrict__ f, int unpack)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= 2L * g.Vh) return;
    int p = (int)(t / g.Vh), i = (int)(t % g.Vh);
    int c[4];
    eo_coords(g, p, i, c);
    long lex = c[0] + (long)g.L[0] * (c[1] + (long)g.L[1] * (c[2] + (long)g.L[2] * c[3]));
    for (int mu = 0; mu < 4; mu++)
        for (int a = 0; a < 8; a++) {
            long ii = ((long)(p * 4 + mu) * 8 + a) * g.Vh + i;
            long cc = (lex * 4 + mu) * 8 + a;
            if (unpack) ((double *)can)[cc] = f[ii];
            else f[ii] = can[cc];
        }
}

__global__ void k_index_maps(Geom g, int32_t *lexeo, int32_t *nbr, int8_t *sign)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= 2L * g.Vh) return;
    int p = (int)(t / g.Vh), i = (int)(t % g.Vh);
    int c[4];
    eo_coords(g, p, i, c);
    lexeo[t] = c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
    for (int mu = 0; mu < 4; mu++)
        for (int b = 0; b < 2; b++) {
            int s;
            int j = eo_neighbour(g, c, mu, b ? -1 : +1, &s);
            nbr[t * 8 + 2 * mu + b] = j;
            sign[t * 8 + 2 * mu + b] = (int8_t)s;
        }
}

}  // namespace

extern "C" int pfmp_create(const int dims[4], int t_bc, void *stream, pfmp_ctx **out)
{
    if (!dims || !out) return PFMP_ERR_ARG;
    *out = nullptr;
    long V = 1;
    for (int m = 0; m < 4; m++) {
        if (dims[m] < 4 || (dims[m] & 1)) return PFMP_ERR_ARG;
        V *= dims[m];
    }
    if (V > 2147483647L) return PFMP_ERR_ARG;   // site indices are int
    if (t_bc != 1 && t_bc != -1) return PFMP_ERR_ARG;
    pfmp_ctx *ctx = new pfmp_ctx();
    for (int m = 0; m < 4; m++) ctx->g.L[m] = dims[m];
    ctx->g.Lh0 = dims[0] / 2;
    ctx->g.V = (int)V;
    ctx->g.Vh = (int)(V / 2);
    ctx->g.tbc = t_bc;
    ctx->g.recon = 0;
    ctx->g.zt = 0;
    // links streamed past the caches once the FP64 gauge field outgrows a good part of
    // the last-level cache (the autotuner may revise this and the visit order)
    ctx->g.stream = 8.0 * gauge_reals(ctx->g) > 128.0 * 1024 * 1024 ? 1 : 0;
    ctx->stream = (hipStream_t)stream;
    ctx->ws = new SolverWS();
    ctx->nblk_red = 1024;
    size_t gb = sizeof(double) * gauge_reals(ctx->g);
    if (hipMalloc(&ctx->U, gb) != hipSuccess || hipMalloc(&ctx->Uf, gb / 2) != hipSuccess ||
        hipMalloc(&ctx->Uh, gb / 4) != hipSuccess ||
        hipMalloc(&ctx->red, sizeof(double) * 64 * 4096) != hipSuccess ||
        hipMalloc(&ctx->scal, sizeof(double) * 8192) != hipSuccess ||

        hipHostMalloc(&ctx->red_host, sizeof(double) * 4096, hipHostMallocDefault) != hipSuccess) {
        pfmp_destroy(ctx);
        return PFMP_ERR_OOM;
    }
    if (noalloc_scratch_init(ctx) != 0) {
        pfmp_destroy(ctx);
        return PFMP_ERR_HIP;
    }
    *out = ctx;
    return 0;
}

extern "C" int pfmp_destroy(pfmp_ctx *ctx)
{
    if (!ctx) return PFMP_ERR_ARG;
    hipStreamSynchronize(ctx->stream);
    hipFree(ctx->U);
    hipFree(ctx->Uf);
    hipFree(ctx->Uh);
    hipFree(ctx->Fhat);
    for (auto &gr : ctx->graphs) hipGraphExecDestroy(gr.exec);
    if (ctx->cap) hipStreamDestroy(ctx->cap);
    hipFree(ctx->red);
    hipFree(ctx->scal);
    if (ctx->red_host) hipHostFree(ctx->red_host);
    for (auto &s : ctx->ops) {
        hipFree(s.clov[0]); hipFree(s.clov[1]);
        hipFree(s.clovf[0]); hipFree(s.clovf[1]);
        hipFree(s.clovh[0]); hipFree(s.clovh[1]);
        hipFree(s.ldpart);
    }
    for (double2 *p : ctx->pool) hipFree(p);
    if (ctx->ws) {
        for (int k = 0; k < kWsSlots; k++) hipFree(ctx->ws->buf[k]);
        delete ctx->ws;
    }
    delete ctx;
    return 0;
}

extern "C" const char *pfmp_last_error(pfmp_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" long long pfmp_field_bytes(pfmp_ctx *ctx, int field, int prec)
{
    if (!ctx) return -1;
    switch (field) {
    case PFMP_FIELD_SPINOR:
        if (prec == PFMP_F64) return 8LL * spinor_reals(ctx->g);
        if (prec == PFMP_F32) return 4LL * spinor_reals(ctx->g);
        if (prec == PFMP_F16) return 2LL * spinor_reals(ctx->g) + 4LL * ctx->g.Vh;
        return -1;
    case PFMP_FIELD_GAUGE: return 8LL * gauge_reals(ctx->g);
    case PFMP_FIELD_MOMENTA: return 8LL * mom_reals(ctx->g);
    }
    return -1;
}

extern "C" int pfmp_index_maps(pfmp_ctx *ctx, int32_t *lex_of_eo, int32_t *nbr, int8_t *sign)
{
    if (!ctx || !lex_of_eo || !nbr || !sign) return ctx ? set_err(ctx, PFMP_ERR_ARG, "index_maps: null") : PFMP_ERR_ARG;
    hipLaunchKernelGGL(k_index_maps, dim3(nblocks(2L * ctx->g.Vh, kBlock)), dim3(kBlock), 0, ctx->stream, ctx->g,
                       lex_of_eo, nbr, sign);
    LAUNCHCHK(ctx);
    return 0;
}

// The links changed: everything derived from them is rebuilt on first use.
int rebuild_gauge_derived(pfmp_ctx *ctx)
{
    ctx->uf_stale = true;
    ctx->fhat_stale = true;
    for (int op = 0; op < PFMP_MAX_OPS; op++)
        if (ctx->ops[op].valid) ctx->ops[op].stale = true;
    return 0;
}

int gauge_f32_ready(pfmp_ctx *ctx)
{
    if (!ctx->uf_stale) return 0;
    long n = gauge_reals(ctx->g) / 2;
    hipLaunchKernelGGL(k_gauge_f32, dim3(nblocks(n, 256)), dim3(256), 0, ctx->stream, (long)ctx->g.Vh, n, ctx->U,
                       ctx->Uf, (__half2 *)ctx->Uh);
    LAUNCHCHK(ctx);
    ctx->uf_stale = false;
    return 0;
}

// per-block maximum over links of max(|U U^dag - 1|_max, |det U - 1|)
__global__ __launch_bounds__(256) void k_su3_dev(Geom g, const double2 *__restrict__ U, double *__restrict__ part)
{
    const long n = 8L * g.Vh;
    double m = 0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const long pm = t / g.Vh, i = t - pm * g.Vh;
        double2 u[9];
        for (int k = 0; k < 9; k++) u[k] = U[(pm * 9 + k) * g.Vh + i];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double2 s = make_double2(a == b ? -1.0 : 0.0, 0.0);
                for (int c = 0; c < 3; c++) cfma(s, u[3 * a + c], cconj(u[3 * b + c]));
                m = fmax(m, fmax(fabs(s.x), fabs(s.y)));
            }
        double2 d = cmul(u[0], csub(cmul(u[4], u[8]), cmul(u[5], u[7])));
        d = csub(d, cmul(u[1], csub(cmul(u[3], u[8]), cmul(u[5], u[6]))));
        d = cadd(d, cmul(u[2], csub(cmul(u[3], u[7]), cmul(u[4], u[6]))));
        m = fmax(m, fmax(fabs(d.x - 1.0), fabs(d.y)));
    }
    __shared__ double sh[4];
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// Links within this distance of SU(3) let the hopping kernels read rows 1, 2 only.
constexpr double kSu3Tol = 1e-12;

static int check_su3(pfmp_ctx *ctx)
{
    const int nb = 256;
    hipLaunchKernelGGL(k_su3_dev, dim3(nb), dim3(256), 0, ctx->stream, ctx->g, ctx->U, ctx->red);
    LAUNCHCHK(ctx);
    std::vector<double> h(nb);
    HIPCHK(ctx, hipMemcpyAsync(h.data(), ctx->red, sizeof(double) * nb, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    double m = 0;
    for (double v : h) m = v > m ? v : m;
    ctx->links_su3 = m <= kSu3Tol;
    ctx->g.recon = ctx->links_su3 && ctx->recon_allowed ? 1 : 0;
    return 0;
}

extern "C" int pfmp_set_gauge(pfmp_ctx *ctx, const void *U_canonical)
{
    if (!ctx || !U_canonical) return ctx ? set_err(ctx, PFMP_ERR_ARG, "set_gauge: null") : PFMP_ERR_ARG;
    hipLaunchKernelGGL(k_pack_gauge, dim3(nblocks(2L * ctx->g.Vh, kBlock)), dim3(kBlock), 0, ctx->stream, ctx->g,
                       (const double2 *)U_canonical, ctx->U, 0);
    LAUNCHCHK(ctx);
    ctx->have_gauge = true;
    int rc = check_su3(ctx);
    return rc ? rc : rebuild_gauge_derived(ctx);
}

extern "C" int pfmp_set_link_reconstruct(pfmp_ctx *ctx, int allow)
{
    if (!ctx) return PFMP_ERR_ARG;
    ctx->recon_allowed = allow != 0;
    ctx->g.recon = ctx->links_su3 && ctx->recon_allowed ? 1 : 0;
    return 0;
}

extern "C" int pfmp_set_site_order(pfmp_ctx *ctx, int zt)
{
    if (!ctx) return PFMP_ERR_ARG;
    if (zt < 0 || (zt > 0 && ctx->g.L[2] % zt != 0))
        return set_err(ctx, PFMP_ERR_ARG, "site order: zt must be 0 or divide the z extent");
    ctx->g.zt = zt;
    return 0;
}

extern "C" int pfmp_set_link_streaming(pfmp_ctx *ctx, int on)
{
    if (!ctx) return PFMP_ERR_ARG;
    ctx->g.stream = on ? 1 : 0;
    return 0;
}

// Time stage 1 + stage 2 of Mhat (slot op, FP64) for every site visit order (memory
// order and each divisor of the z extent up to 16) with cached and with streaming
// link loads; keep the fastest.
extern "C" int pfmp_autotune(pfmp_ctx *ctx, int op, pfmp_tuning *out)
{
    if (!ctx) return PFMP_ERR_ARG;
    int rc = op_ready(ctx, op);
    if (rc) return rc;
    double2 *in = pool_get(ctx, 2400), *o = pool_get(ctx, 2401), *tmp = pool_get(ctx, 2402);
    if (!in || !o || !tmp) return set_err(ctx, PFMP_ERR_OOM, "autotune workspace");
    HIPCHK(ctx, hipMemsetAsync(in, 0, sizeof(double) * spinor_reals(ctx->g), ctx->stream));
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    const Geom keep = ctx->g;
    double best = 1e30;
    int bzt = keep.zt, bst = keep.stream;
    const int reps = 10;
    for (int st = 0; st < 2; st++)
        for (int zt = 0; zt <= 16 && zt <= keep.L[2]; zt++) {
            if (zt == 1 || (zt > 0 && keep.L[2] % zt != 0)) continue;
            ctx->g.zt = zt;
            ctx->g.stream = st;
            for (int k = 0; k < 2; k++)
                if ((rc = op_apply_M(ctx, op, 0, in, o, tmp, nullptr))) break;
            if (!rc) rc = hipEventRecord(e0, ctx->stream) == hipSuccess ? 0 : set_err(ctx, PFMP_ERR_HIP, "event");
            for (int k = 0; k < reps && !rc; k++) rc = op_apply_M(ctx, op, 0, in, o, tmp, nullptr);
            if (!rc) rc = hipEventRecord(e1, ctx->stream) == hipSuccess ? 0 : set_err(ctx, PFMP_ERR_HIP, "event");
            float ms = 0;
            if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = set_err(ctx, PFMP_ERR_HIP, "autotune timing");
            if (rc) break;
            const double us = 1e3 * ms / reps;
            if (us < best) {
                best = us;
                bzt = zt;
                bst = st;
            }
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    ctx->g = keep;
    if (rc) return rc;
    ctx->g.zt = bzt;
    ctx->g.stream = bst;
    if (out) {
        out->zt = bzt;
        out->stream = bst;
        out->us_Mhat = best;
    }
    return 0;
}

extern "C" int pfmp_get_link_reconstruct(pfmp_ctx *ctx, int *active)
{
    if (!ctx || !active) return ctx ? set_err(ctx, PFMP_ERR_ARG, "get_link_reconstruct: null") : PFMP_ERR_ARG;
    *active = ctx->g.recon;
    return 0;
}

extern "C" int pfmp_get_gauge(pfmp_ctx *ctx, void *U_canonical)
{
    if (!ctx || !U_canonical) return ctx ? set_err(ctx, PFMP_ERR_ARG, "get_gauge: null") : PFMP_ERR_ARG;
    if (!ctx->have_gauge) return set_err(ctx, PFMP_ERR_STATE, "no gauge field set");
    hipLaunchKernelGGL(k_pack_gauge, dim3(nblocks(2L * ctx->g.Vh, kBlock)), dim3(kBlock), 0, ctx->stream, ctx->g,
                       (const double2 *)U_canonical, ctx->U, 1);
    LAUNCHCHK(ctx);
    return 0;
}

extern "C" int pfmp_set_operator(pfmp_ctx *ctx, int op, double kappa, double csw)
{
    if (!ctx) return PFMP_ERR_ARG;
    if (op < 0 || op >= PFMP_MAX_OPS) return set_err(ctx, PFMP_ERR_ARG, "operator slot out of range");
    if (!ctx->have_gauge) return set_err(ctx, PFMP_ERR_STATE, "set_operator needs a gauge field");
    OpSlot &s = ctx->ops[op];
    s.kappa = kappa;
    s.csw = csw;
    if (!s.clov[0]) {
        size_t b = sizeof(double) * clover_reals(ctx->g);
        if (hipMalloc(&s.clov[0], b) != hipSuccess || hipMalloc(&s.clov[1], b) != hipSuccess ||
            hipMalloc(&s.clovf[0], b / 2) != hipSuccess || hipMalloc(&s.clovf[1], b / 2) != hipSuccess ||
            hipMalloc(&s.clovh[0], b / 4) != hipSuccess || hipMalloc(&s.clovh[1], b / 4) != hipSuccess)
            return set_err(ctx, PFMP_ERR_OOM, "clover fields");
    }
    s.valid = true;
    int rc = clover_build(ctx, op);
    if (!rc) rc = clover_logdet(ctx, op);   // positivity checked once, synchronously
    if (rc) s.valid = false;
    return rc;
}

extern "C" int pfmp_pack_spinor(pfmp_ctx *ctx, const void *canonical, void *internal, int prec)
{
    if (!ctx || !canonical || !internal) return ctx ? set_err(ctx, PFMP_ERR_ARG, "pack_spinor: null") : PFMP_ERR_ARG;
    dim3 grid(nblocks(12L * ctx->g.Vh, 256)), block(256);
    if (prec == PFMP_F64)
        hipLaunchKernelGGL((k_pack_spinor<double2>), grid, block, 0, ctx->stream, ctx->g.Vh,
                           (const double2 *)canonical, (double2 *)internal, 0);
    else if (prec == PFMP_F32)
        hipLaunchKernelGGL((k_pack_spinor<float2>), grid, block, 0, ctx->stream, ctx->g.Vh,
                           (const double2 *)canonical, (float2 *)internal, 0);
    else
        return set_err(ctx, PFMP_ERR_ARG, "pack_spinor: unsupported precision");
    LAUNCHCHK(ctx);
    return 0;
}

extern "C" int pfmp_unpack_spinor(pfmp_ctx *ctx, const void *internal, void *canonical, int prec)
{
    if (!ctx || !canonical || !internal) return ctx ? set_err(ctx, PFMP_ERR_ARG, "unpack_spinor: null") : PFMP_ERR_ARG;
    dim3 grid(nblocks(12L * ctx->g.Vh, 256)), block(256);
    if (prec == PFMP_F64)
        hipLaunchKernelGGL((k_pack_spinor<double2>), grid, block, 0, ctx->stream, ctx->g.Vh,
                           (const double2 *)canonical, (double2 *)internal, 1);
    else if (prec == PFMP_F32)
        hipLaunchKernelGGL((k_pack_spinor<float2>), grid, block, 0, ctx->stream, ctx->g.Vh,
                           (const double2 *)canonical, (float2 *)internal, 1);
    else
        return set_err(ctx, PFMP_ERR_ARG, "unpack_spinor: unsupported precision");
    LAUNCHCHK(ctx);
    return 0;
}

extern "C" int pfmp_pack_momenta(pfmp_ctx *ctx, const double *canonical, double *internal)
{
    if (!ctx || !canonical || !internal) return ctx ? set_err(ctx, PFMP_ERR_ARG, "pack_momenta: null") : PFMP_ERR_ARG;
    hipLaunchKernelGGL(k_pack_mom, dim3(nblocks(2L * ctx->g.Vh, kBlock)), dim3(kBlock), 0, ctx->stream, ctx->g,
                       canonical, internal, 0);
    LAUNCHCHK(ctx);
    return 0;
}

extern "C" int pfmp_unpack_momenta(pfmp_ctx *ctx, const double *internal, double *canonical)
{
    if (!ctx || !canonical || !internal) return ctx ? set_err(ctx, PFMP_ERR_ARG, "unpack_momenta: null") : PFMP_ERR_ARG;
    hipLaunchKernelGGL(k_pack_mom, dim3(nblocks(2L * ctx->g.Vh, kBlock)), dim3(kBlock), 0, ctx->stream, ctx->g,
                       canonical, (double *)internal, 1);
    LAUNCHCHK(ctx);
    return 0;
}
