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

// Full 6x6 block b (row-major) of A at site c.
__device__ void clover_block_full(const M3 *F, double kc, int b, double2 *A)
{
    double s = b == 0 ? 1.0 : -1.0;
    // plane order: 0:(01) 1:(02) 2:(03) 3:(12) 4:(13) 5:(23)
    M3 Gx = m3_sub(m3_scale(F[2], s), F[3]);
    M3 Gy = m3_add(m3_scale(F[4], s), F[1]);
    M3 Gz = m3_sub(m3_scale(F[5], s), F[0]);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            int k = 3 * i + j;
            double2 gz = Gz.e[k];
            double2 up = csub(Gx.e[k], ctimesi(Gy.e[k]));   // Gx - i Gy
            double2 lo = cadd(Gx.e[k], ctimesi(Gy.e[k]));   // Gx + i Gy
            // i kc * block
            A[i * 6 + j] = cscale(ctimesi(gz), kc);
            A[i * 6 + 3 + j] = cscale(ctimesi(up), kc);
            A[(3 + i) * 6 + j] = cscale(ctimesi(lo), kc);
            A[(3 + i) * 6 + 3 + j] = cscale(ctimesi(gz), -kc);
        }
    for (int i = 0; i < 6; i++) A[i * 6 + i].x += 1.0;
}

// In-place Cholesky inverse of a 6x6 Hermitian positive matrix; returns ln det, or
// NaN when a pivot is not positive.
__device__ double herm6_inverse(double2 *A)
{
    double2 L[36];
    double ld = 0;
    for (int k = 0; k < 36; k++) L[k] = make_double2(0, 0);
    for (int j = 0; j < 6; j++) {
        double d = A[j * 6 + j].x;
        for (int k = 0; k < j; k++) d -= L[j * 6 + k].x * L[j * 6 + k].x + L[j * 6 + k].y * L[j * 6 + k].y;
        if (!(d > 0)) return __builtin_nan("");
        double ljj = sqrt(d);
        ld += 2.0 * log(ljj);
        L[j * 6 + j] = make_double2(ljj, 0);
        for (int i = j + 1; i < 6; i++) {
            double2 s = A[i * 6 + j];
            for (int k = 0; k < j; k++) s = csub(s, cmul(L[i * 6 + k], cconj(L[j * 6 + k])));
            L[i * 6 + j] = cscale(s, 1.0 / ljj);
        }
    }
    // W = L^-1 (lower triangular)
    double2 W[36];
    for (int k = 0; k < 36; k++) W[k] = make_double2(0, 0);
    for (int i = 0; i < 6; i++) {
        W[i * 6 + i] = make_double2(1.0 / L[i * 6 + i].x, 0);
        for (int j = 0; j < i; j++) {
            double2 s = make_double2(0, 0);
            for (int k = j; k < i; k++) cfma(s, L[i * 6 + k], W[k * 6 + j]);
            W[i * 6 + j] = cscale(s, -1.0 / L[i * 6 + i].x);
        }
    }
    // A^-1 = W^dag W
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 6; j++) {
            double2 s = make_double2(0, 0);
            int k0 = i > j ? i : j;
            for (int k = k0; k < 6; k++) cfmac(s, W[k * 6 + i], W[k * 6 + j]);
            A[i * 6 + j] = s;
        }
    return ld;
}

__global__ __launch_bounds__(kBlock) void k_clover_build(Geom g, int parity, const double2 *__restrict__ U,
                                                         double kc, double *__restrict__ out,
                                                         double *__restrict__ ld_partials, int *__restrict__ bad)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double ld = 0;
    if (i < g.Vh) {
        int c[4];
        eo_coords(g, parity, i, c);
        M3 F[6];
        int p = 0;
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++, p++) F[p] = fhat(g, U, c, mu, nu);
        double2 *off = reinterpret_cast<double2 *>(out + 12L * g.Vh);
        for (int b = 0; b < 2; b++) {
            double2 A[36];
            clover_block_full(F, kc, b, A);
            if (parity == 1) {
                double l = herm6_inverse(A);
                if (l != l) { *bad = 1; l = 0; }
                ld += l;
            }
            for (int k = 0; k < 6; k++) out[(long)(b * 6 + k) * g.Vh + i] = A[k * 6 + k].x;
            int m = 0;
            for (int r = 0; r < 6; r++)
                for (int q = r + 1; q < 6; q++, m++) off[(long)(b * 15 + m) * g.Vh + i] = A[r * 6 + q];
        }
    }
    if (parity == 1) {
        __shared__ double sh[kBlock / 64];
        for (int o = 32; o > 0; o >>= 1) ld += __shfl_down(ld, o, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = ld;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0;
            for (int k = 0; k < kBlock / 64; k++) s += sh[k];
            ld_partials[blockIdx.x] = s;
        }
    }
}

__global__ void k_to_f32(long n, const double *__restrict__ a, float *__restrict__ b)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) b[t] = (float)a[t];
}

}  // namespace

// Rebuild the clover fields of slot op on the current links.  No host
// synchronisation: the per-block ln det partials and the positivity flag stay on
// the device until clover_logdet() needs them.
int clover_build(pfmp_ctx *ctx, int op)
{
    OpSlot &s = ctx->ops[op];
    const Geom &g = ctx->g;
    s.logdet_odd = 0;
    s.ld_dirty = false;
    if (s.csw == 0) return 0;
    const int nb = nblocks(g.Vh, kBlock);
    if (!s.ldpart && hipMalloc(&s.ldpart, sizeof(double) * nb) != hipSuccess)
        return set_err(ctx, PFMP_ERR_OOM, "clover workspace");
    int *bad = (int *)(ctx->scal + 8000) + op;
    HIPCHK(ctx, hipMemsetAsync(bad, 0, sizeof(int), ctx->stream));
    const double kc = s.kappa * s.csw;
    for (int p = 0; p < 2; p++) {
        hipLaunchKernelGGL(k_clover_build, dim3(nb), dim3(kBlock), 0, ctx->stream, g, p, ctx->U, kc, s.clov[p],
                           s.ldpart, bad);
        LAUNCHCHK(ctx);
        long n = clover_reals(g);
        hipLaunchKernelGGL(k_to_f32, dim3(nblocks(n, 256)), dim3(256), 0, ctx->stream, n, s.clov[p], s.clovf[p]);
        LAUNCHCHK(ctx);
    }
    s.ld_dirty = true;
    return 0;
}

// Sum the ln det A_oo partials of slot op (synchronises) and check positivity.
int clover_logdet(pfmp_ctx *ctx, int op)
{
    OpSlot &s = ctx->ops[op];
    if (!s.ld_dirty) return 0;
    const int nb = nblocks(ctx->g.Vh, kBlock);
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
    if (!ctx->ops[op].valid) return set_err(ctx, PFMP_ERR_STATE, "operator slot not configured");
    int rc = clover_logdet(ctx, op);
    if (rc) return rc;
    *out = -2.0 * ctx->ops[op].logdet_odd;
    return 0;
}
