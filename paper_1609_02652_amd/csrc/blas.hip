// blas.hip -- BLAS-1 on internal FP64 spinors with deterministic FP64 reductions.
//
// A reduction is two launches: a grid kernel writes one partial per block (wave
// shuffles, then LDS across the block's waves, fixed order), and a single-block
// kernel sums the partials in a fixed strided order.  No atomics: results are
// bitwise reproducible run to run.
#include <vector>

#include "internal.h"

namespace {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

template <int NB>
__device__ __forceinline__ void block_store(double v, double *out)
{
    __shared__ double sh[NB / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
        for (int k = 0; k < NB / 64; k++) s += sh[k];
        *out = s;
    }
    __syncthreads();
}

// grid-stride partial sums of <a, b> (complex): partials[2*block + {0,1}]
__global__ __launch_bounds__(kRedBlock) void k_dot(const double2 *__restrict__ a, const double2 *__restrict__ b,
                                                   long n, double *__restrict__ partials)
{
    double re = 0, im = 0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        double2 x = a[t], y = b[t];
        re += x.x * y.x + x.y * y.y;
        im += x.x * y.y - x.y * y.x;
    }
    block_store<kRedBlock>(re, partials + 2 * blockIdx.x);
    block_store<kRedBlock>(im, partials + 2 * blockIdx.x + 1);
}

__global__ __launch_bounds__(kRedBlock) void k_norm2(const double2 *__restrict__ a, long n,
                                                     double *__restrict__ partials)
{
    double s = 0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        double2 x = a[t];
        s += x.x * x.x + x.y * x.y;
    }
    block_store<kRedBlock>(s, partials + blockIdx.x);
}

// out[v] = sum_k partials[k * nvals + v], one block
__global__ __launch_bounds__(kRedBlock) void k_finish(const double *__restrict__ partials, int nparts, int nvals,
                                                      double *__restrict__ out)
{
    for (int v = 0; v < nvals; v++) {
        double s = 0;
        for (int k = threadIdx.x; k < nparts; k += blockDim.x) s += partials[(long)k * nvals + v];
        block_store<kRedBlock>(s, out + v);
    }
}

__global__ void k_axpby(long n, double2 al, const double2 *__restrict__ x, double2 be, double2 *__restrict__ y)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) y[t] = cadd(cmul(al, x[t]), cmul(be, y[t]));
}

}  // namespace

template <typename A, typename B>
__global__ void k_convert(long n, const A *__restrict__ x, B *__restrict__ y)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) y[t] = mk<B>((decltype(B::x))x[t].x, (decltype(B::x))x[t].y);
}

int launch_dot(pfmp_ctx *ctx, const double2 *a, const double2 *b, long n, double *partials)
{
    hipLaunchKernelGGL(k_dot, dim3(ctx->nblk_red), dim3(kRedBlock), 0, ctx->stream, a, b, n, partials);
    LAUNCHCHK(ctx);
    return 0;
}

int launch_norm2(pfmp_ctx *ctx, const double2 *a, long n, double *partials)
{
    hipLaunchKernelGGL(k_norm2, dim3(ctx->nblk_red), dim3(kRedBlock), 0, ctx->stream, a, n, partials);
    LAUNCHCHK(ctx);
    return 0;
}

// Sum nparts partial records of nvals values into device scalars dev_out (if
// non-null) and, when host_out is non-null, copy them to the host (synchronises).
int red_finish_dev(pfmp_ctx *ctx, const double *partials, int nparts, int nvals, double *dev_out)
{
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kRedBlock), 0, ctx->stream, partials, nparts, nvals, dev_out);
    LAUNCHCHK(ctx);
    return 0;
}

int red_finish(pfmp_ctx *ctx, const double *partials, int nparts, int nvals, double *host_out)
{
    double *dev = ctx->scal + 7000;
    int rc = red_finish_dev(ctx, partials, nparts, nvals, dev);
    if (rc) return rc;
    HIPCHK(ctx, hipMemcpyAsync(ctx->red_host, dev, sizeof(double) * nvals, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int v = 0; v < nvals; v++) host_out[v] = ctx->red_host[v];
    return 0;
}

extern "C" int pfmp_dot(pfmp_ctx *ctx, const void *a, const void *b, double out[2])
{
    if (!ctx || !a || !b || !out) return ctx ? set_err(ctx, PFMP_ERR_ARG, "dot: null") : PFMP_ERR_ARG;
    long n = 12L * ctx->g.Vh;
    int rc = launch_dot(ctx, (const double2 *)a, (const double2 *)b, n, ctx->red);
    if (rc) return rc;
    return red_finish(ctx, ctx->red, ctx->nblk_red, 2, out);
}

extern "C" int pfmp_axpby(pfmp_ctx *ctx, const double alpha[2], const void *x, const double beta[2], void *y)
{
    if (!ctx || !alpha || !beta || !x || !y) return ctx ? set_err(ctx, PFMP_ERR_ARG, "axpby: null") : PFMP_ERR_ARG;
    long n = 12L * ctx->g.Vh;
    hipLaunchKernelGGL(k_axpby, dim3(nblocks(n, 256)), dim3(256), 0, ctx->stream, n,
                       make_double2(alpha[0], alpha[1]), (const double2 *)x, make_double2(beta[0], beta[1]),
                       (double2 *)y);
    LAUNCHCHK(ctx);
    return 0;
}

extern "C" int pfmp_convert_spinor(pfmp_ctx *ctx, const void *in, int prec_in, void *out, int prec_out)
{
    if (!ctx || !in || !out) return ctx ? set_err(ctx, PFMP_ERR_ARG, "convert_spinor: null") : PFMP_ERR_ARG;
    const bool ok_in = prec_in == PFMP_F64 || prec_in == PFMP_F32, ok_out = prec_out == PFMP_F64 || prec_out == PFMP_F32;
    if (!ok_in || !ok_out) return set_err(ctx, PFMP_ERR_ARG, "convert_spinor: FP64 or FP32 fields only");
    long n = 12L * ctx->g.Vh;
    dim3 grid(nblocks(n, 256)), block(256);
    if (prec_in == PFMP_F64 && prec_out == PFMP_F32)
        hipLaunchKernelGGL((k_convert<double2, float2>), grid, block, 0, ctx->stream, n, (const double2 *)in, (float2 *)out);
    else if (prec_in == PFMP_F32 && prec_out == PFMP_F64)
        hipLaunchKernelGGL((k_convert<float2, double2>), grid, block, 0, ctx->stream, n, (const float2 *)in, (double2 *)out);
    else
        HIPCHK(ctx, hipMemcpyAsync(out, in, n * (prec_in == PFMP_F64 ? sizeof(double2) : sizeof(float2)),
                                   hipMemcpyDeviceToDevice, ctx->stream));
    LAUNCHCHK(ctx);
    return 0;
}
