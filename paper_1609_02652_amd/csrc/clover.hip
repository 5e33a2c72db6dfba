// clover.hip -- clover term A = 1 + i kappa c_sw sum_{mu<nu} sigma_mu_nu Fhat_mu_nu.
//
// Fhat_mu_nu = (Q - Q^dag)/8 with Q the sum of the four leaves at x in the
// (mu,nu) plane.  In the chiral basis sigma_mu_nu is block diagonal; with the
// plane order p = (01)(02)(03)(12)(13)(23) and s = +1 (spins 0,1) / -1 (spins 2,3):
//   sigma_p = -s_z, +s_y, +s_x, -s_x, +s_y, +s_z   on the upper block
//   sigma_p = -s_z, +s_y, -s_x, -s_x, -s_y, -s_z   on the lower block
// so each block is 1 + i kappa c_sw [[Gz, Gx - i Gy], [Gx + i Gy, -Gz]] with
//   Gx = s F_03 - F_12,  Gy = s F_13 + F_02,  Gz = s F_23 - F_01.
// Even sites store A (diagonal + upper triangle of each 6x6 block); odd sites store
// A^-1 from a Cholesky factorisation, whose pivots also give ln det A.
#include <hip/hip_fp16.h>

#include "hop.h"
#include "su3.h"

namespace {

// Q_mu_nu(x): sum of the four leaves, all traversed in the same sense.
__device__ M3 clover_leaves(const Geom &g, const double2 *__restrict__ U, const int *c, int mu, int nu)
{
    int xpm[4], xpn[4], xmm[4], xmn[4], xpnmm[4], xmmmn[4], xmnpm[4];
    shifted(g, c, mu, +1, xpm);
    shifted(g, c, nu, +1, xpn);
    shifted(g, c, mu, -1, xmm);
    shifted(g, c, nu, -1, xmn);
    shifted(g, xpn, mu, -1, xpnmm);
    shifted(g, xmm, nu, -1, xmmmn);
    shifted(g, xmn, mu, +1, xmnpm);
    M3 Umu_x = link_at(g, U, c, mu), Unu_x = link_at(g, U, c, nu);
    // leaf 0: U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
    M3 q = m3_mul_nd(m3_mul(Umu_x, link_at(g, U, xpm, nu)), m3_mul(Unu_x, link_at(g, U, xpn, mu)));
    // leaf 1: U_nu(x) U_mu(x+nu-mu)^dag U_nu(x-mu)^dag U_mu(x-mu)
    M3 a = m3_mul_nd(Unu_x, link_at(g, U, xpnmm, mu));
    M3 b = m3_mul_dn(link_at(g, U, xmm, nu), link_at(g, U, xmm, mu));
    q = m3_add(q, m3_mul(a, b));
    // leaf 2: U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu)
    a = m3_mul_dn(m3_mul(link_at(g, U, xmmmn, nu), link_at(g, U, xmm, mu)), link_at(g, U, xmmmn, mu));
    q = m3_add(q, m3_mul(a, link_at(g, U, xmn, nu)));
    // leaf 3: U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^dag
    a = m3_mul_dn(link_at(g, U, xmn, nu), link_at(g, U, xmn, mu));
    q = m3_add(q, m3_mul_nd(m3_mul(a, link_at(g, U, xmnpm, nu)), Umu_x));
    return q;
}

__device__ M3 fhat(const Geom &g, const double2 *__restrict__ U, const int *c, int mu, int nu)
{
    M3 q = clover_leaves(g, U, c, mu, nu);
    return m3_scale(m3_sub(q, m3_dag(q)), 0.125);
}

// F-hat of one plane at one site, for both parities: thread (p, plane, i), sites fastest.
__global__ __launch_bounds__(kBlock) void k_fhat(Geom g, const double2 *__restrict__ U, double2 *__restrict__ Fh)
{
    long t = xcd_lane(12L * g.Vh);   // XCD-aware order: the leaves' link gathers through one L2
    if (t >= 12L * g.Vh) return;
    const int pp = (int)(t / g.Vh), i = (int)(t - (long)pp * g.Vh);
    const int p = pp / 6, pl = pp - 6 * p;
    const int mu = pl < 3 ? 0 : (pl < 5 ? 1 : 2);
    const int nu = pl < 3 ? pl + 1 : (pl < 5 ? pl - 1 : 3);
    int c[4];
    eo_coords(g, p, i, c);
    M3 f = fhat(g, U, c, mu, nu);
    double2 *o = Fh + ((long)pp * 9) * g.Vh + i;
    for (int k = 0; k < 9; k++) o[(long)k * g.Vh] = f.e[k];
}

__device__ __forceinline__ constexpr int tri(int r, int c) { return r * (r + 1) / 2 + c; }   // c <= r

// FP16 copy of a clover field (round to nearest), for the FP16-storage inner solver:
// thread t = 2 i + b packs the FP32 record of block b of site i (6 diagonal reals, 15
// complex entries) into its 72-byte record of 6 H3 at h[t * 6]
__global__ void k_clover_half(long Vh, const float *__restrict__ a, H3 *__restrict__ h)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= 2 * Vh) return;
    float f[36];
    const float4 *rf = reinterpret_cast<const float4 *>(a) + t * 9;
#pragma unroll
    for (int u = 0; u < 9; u++) {
        const float4 v = rf[u];
        f[4 * u] = v.x; f[4 * u + 1] = v.y; f[4 * u + 2] = v.z; f[4 * u + 3] = v.w;
    }
    H3 q[6];
#pragma unroll
    for (int k = 0; k < 3; k++) q[0].v[k] = __floats2half2_rn(f[2 * k], f[2 * k + 1]);
#pragma unroll
    for (int m = 0; m < 15; m++) q[1 + m / 3].v[m % 3] = __floats2half2_rn(f[6 + 2 * m], f[7 + 2 * m]);
    H3 *rec = h + t * 6;
#pragma unroll
    for (int u = 0; u < 6; u++) rec[u] = q[u];
}

// Chiral block b of A at parity p from F-hat: thread (b, i).  INV = 0 stores A
// (even sites); INV = 1 stores A^-1 from a packed Cholesky factorisation and sums
// ln det A into per-block partials (odd sites).  Storage: 6 real diagonal entries
// and the 15 upper off-diagonal entries (row-major) of each block; FP64 in planes (12
// diagonal planes [b * 6 + k][Vh], 30 complex planes [b * 15 + m][Vh]), FP32 as one record
// of 36 floats per block and site at (2 i + b) * 36 (nine 16-byte loads).
// Each block is 1 + i kappa c_sw [[Gz, Gx - i Gy], [Gx + i Gy, -Gz]] with
// Gx = s F_03 - F_12, Gy = s F_13 + F_02, Gz = s F_23 - F_01, s = +1 (b = 0) / -1 (b = 1).
template <int INV>
__global__ __launch_bounds__(kBlock) void k_clover_blocks(Geom g, int p, const double2 *__restrict__ Fh, double kc,
                                                          double *__restrict__ out, float *__restrict__ outf,
                                                          double *__restrict__ ld_partials, int *__restrict__ bad)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    double ld = 0;
    if (t < 2L * g.Vh) {
        const int b = (int)(t / g.Vh), i = (int)(t - (long)b * g.Vh);
        const long Vh = g.Vh;
        const double s = b == 0 ? 1.0 : -1.0;
        const double2 *F = Fh + ((long)p * 6 * 9) * Vh + i;
        auto fe = [&](int pl, int k) { return F[((long)pl * 9 + k) * Vh]; };
        double2 a[21];   // lower triangle, row-major
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
            for (int c = 0; c <= r; c++) {
                int k = 3 * r + c;
                double2 gz = csub(cscale(fe(5, k), s), fe(0, k));
                a[tri(r, c)] = cscale(ctimesi(gz), kc);
                a[tri(3 + r, 3 + c)] = cscale(ctimesi(gz), -kc);
            }
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
            for (int c = 0; c < 3; c++) {
                int k = 3 * r + c;
                double2 gx = csub(cscale(fe(2, k), s), fe(3, k));
                double2 gy = cadd(cscale(fe(4, k), s), fe(1, k));
                a[tri(3 + r, c)] = cscale(ctimesi(cadd(gx, ctimesi(gy))), kc);
            }
#pragma unroll
        for (int r = 0; r < 6; r++) a[tri(r, r)] = make_double2(a[tri(r, r)].x + 1.0, 0.0);

        double *dg = out + (long)(b * 6) * Vh + i;
        double2 *off = reinterpret_cast<double2 *>(out + 12L * Vh) + (long)(b * 15) * Vh + i;
        float rec[36];   // the FP32 record of the block: 6 diagonal reals, 15 complex entries
        if (!INV) {
            int m = 0;
#pragma unroll
            for (int r = 0; r < 6; r++) {
                dg[(long)r * Vh] = a[tri(r, r)].x;
                rec[r] = (float)a[tri(r, r)].x;
#pragma unroll
                for (int q = r + 1; q < 6; q++, m++) {
                    double2 v = cconj(a[tri(q, r)]);
                    off[(long)m * Vh] = v;
                    rec[6 + 2 * m] = (float)v.x;
                    rec[7 + 2 * m] = (float)v.y;
                }
            }
        } else {
            // A = L L^dag in place
            bool ok = true;
#pragma unroll
            for (int j = 0; j < 6; j++) {
                double d = a[tri(j, j)].x;
#pragma unroll
                for (int k = 0; k < j; k++) d -= a[tri(j, k)].x * a[tri(j, k)].x + a[tri(j, k)].y * a[tri(j, k)].y;
                ok = ok && d > 0;
                double ljj = sqrt(d > 0 ? d : 1.0);
                ld += 2.0 * log(ljj);
                a[tri(j, j)] = make_double2(ljj, 0.0);
                const double inv = 1.0 / ljj;
#pragma unroll
                for (int r = j + 1; r < 6; r++) {
                    double2 v = a[tri(r, j)];
#pragma unroll
                    for (int k = 0; k < j; k++) v = csub(v, cmul(a[tri(r, k)], cconj(a[tri(j, k)])));
                    a[tri(r, j)] = cscale(v, inv);
                }
            }
            if (!ok) {
                *bad = 1;
                ld = 0;
            }
            // column c of A^-1: L y = e_c, then L^dag x = y; keep rows r <= c
#pragma unroll
            for (int c = 0; c < 6; c++) {
                double2 y[6];
#pragma unroll
                for (int r = 0; r < 6; r++) {
                    if (r < c) {
                        y[r] = make_double2(0, 0);
                        continue;
                    }
                    double2 v = make_double2(r == c ? 1.0 : 0.0, 0.0);
#pragma unroll
                    for (int k = c; k < r; k++) v = csub(v, cmul(a[tri(r, k)], y[k]));
                    y[r] = cscale(v, 1.0 / a[tri(r, r)].x);
                }
#pragma unroll
                for (int r = 5; r >= 0; r--) {
                    double2 v = y[r];
#pragma unroll
                    for (int k = r + 1; k < 6; k++) v = csub(v, cmul(cconj(a[tri(k, r)]), y[k]));
                    y[r] = cscale(v, 1.0 / a[tri(r, r)].x);
                }
                dg[(long)c * Vh] = y[c].x;
                rec[c] = (float)y[c].x;
#pragma unroll
                for (int r = 0; r < c; r++) {
                    const int m = r * 5 - r * (r - 1) / 2 + (c - r - 1);   // index of (r, c), r < c
                    off[(long)m * Vh] = y[r];
                    rec[6 + 2 * m] = (float)y[r].x;
                    rec[7 + 2 * m] = (float)y[r].y;
                }
            }
        }
        float4 *rf = reinterpret_cast<float4 *>(outf) + (2L * i + b) * 9;
#pragma unroll
        for (int u = 0; u < 9; u++) rf[u] = make_float4(rec[4 * u], rec[4 * u + 1], rec[4 * u + 2], rec[4 * u + 3]);
    }
    if (INV) {
        __shared__ double sh[kBlock / 64];
        for (int o = 32; o > 0; o >>= 1) ld += __shfl_down(ld, o, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = ld;
        __syncthreads();
        if (threadIdx.x == 0) {
            double sum = 0;
            for (int k = 0; k < kBlock / 64; k++) sum += sh[k];
            ld_partials[blockIdx.x] = sum;
        }
    }
}

}  // namespace

static int fhat_ready(pfmp_ctx *ctx)
{
    if (!ctx->fhat_stale) return 0;
    const Geom &g = ctx->g;
    if (!ctx->Fhat && hipMalloc(&ctx->Fhat, sizeof(double2) * 108L * g.Vh) != hipSuccess) {
        ctx->Fhat = nullptr;
        return set_err(ctx, PFMP_ERR_OOM, "clover field strength");
    }
    hipLaunchKernelGGL(k_fhat, dim3(nblocks_site(12L * g.Vh)), dim3(kBlock), 0, ctx->stream, g, ctx->U, ctx->Fhat);
    LAUNCHCHK(ctx);
    ctx->fhat_stale = false;
    return 0;
}

// Rebuild the clover fields of slot op on the current links (F-hat shared by all
// slots).  No host synchronisation: the ln det partials and the positivity flag
// stay on the device until clover_logdet() needs them.
int clover_build(pfmp_ctx *ctx, int op)
{
    OpSlot &s = ctx->ops[op];
    const Geom &g = ctx->g;
    s.logdet_odd = 0;
    s.ld_dirty = false;
    s.stale = false;
    if (s.csw == 0) return 0;
    int rc = fhat_ready(ctx);
    if (rc) return rc;
    const int nb = nblocks(2L * g.Vh, kBlock);
    if (!s.ldpart && hipMalloc(&s.ldpart, sizeof(double) * nb) != hipSuccess) {
        s.ldpart = nullptr;
        return set_err(ctx, PFMP_ERR_OOM, "clover workspace");
    }
    int *bad = (int *)(ctx->scal + 8000) + op;
    HIPCHK(ctx, hipMemsetAsync(bad, 0, sizeof(int), ctx->stream));
    const double kc = s.kappa * s.csw;
    hipLaunchKernelGGL(k_clover_blocks<0>, dim3(nb), dim3(kBlock), 0, ctx->stream, g, 0, ctx->Fhat, kc, s.clov[0],
                       s.clovf[0], s.ldpart, bad);
    LAUNCHCHK(ctx);
    hipLaunchKernelGGL(k_clover_blocks<1>, dim3(nb), dim3(kBlock), 0, ctx->stream, g, 1, ctx->Fhat, kc, s.clov[1],
                       s.clovf[1], s.ldpart, bad);
    LAUNCHCHK(ctx);
    for (int p = 0; p < 2; p++)
        hipLaunchKernelGGL(k_clover_half, dim3(nblocks(2L * g.Vh, 256)), dim3(256), 0, ctx->stream, (long)g.Vh,
                           s.clovf[p], (H3 *)s.clovh[p]);
    LAUNCHCHK(ctx);
    s.ld_dirty = true;
    return 0;
}

// Slot op configured and its clover fields current for the present links.
int op_ready(pfmp_ctx *ctx, int op)
{
    if (op < 0 || op >= PFMP_MAX_OPS) return set_err(ctx, PFMP_ERR_ARG, "operator slot out of range");
    if (!ctx->have_gauge) return set_err(ctx, PFMP_ERR_STATE, "no gauge field set");
    if (!ctx->ops[op].valid) return set_err(ctx, PFMP_ERR_STATE, "operator slot not configured");
    return ctx->ops[op].stale ? clover_build(ctx, op) : 0;
}

// Sum the ln det A_oo partials of slot op (synchronises) and check positivity.
int clover_logdet(pfmp_ctx *ctx, int op)
{
    OpSlot &s = ctx->ops[op];
    if (!s.ld_dirty) return 0;
    const int nb = nblocks(2L * ctx->g.Vh, kBlock);
    std::vector<double> h(nb);
    int hbad = 0;
    HIPCHK(ctx, hipMemcpyAsync(h.data(), s.ldpart, sizeof(double) * nb, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(&hbad, (int *)(ctx->scal + 8000) + op, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (hbad) return set_err(ctx, PFMP_ERR_ARG, "clover term A_oo is not positive definite");
    double t = 0;
    for (double v : h) t += v;
    s.logdet_odd = t;
    s.ld_dirty = false;
    return 0;
}

extern "C" int pfmp_logdet_action(pfmp_ctx *ctx, int op, double *out)
{
    if (!ctx || !out || op < 0 || op >= PFMP_MAX_OPS) return ctx ? set_err(ctx, PFMP_ERR_ARG, "logdet_action") : PFMP_ERR_ARG;
    int rc = op_ready(ctx, op);
    if (!rc) rc = clover_logdet(ctx, op);
    if (rc) return rc;
    *out = -2.0 * ctx->ops[op].logdet_odd;
    return 0;
}
