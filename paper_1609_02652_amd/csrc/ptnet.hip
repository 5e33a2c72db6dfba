// ptnet.hip -- learned gauge-covariant preconditioner for a flexible CG.
//
// Network (2 parallel-transport convolution layers, 12 complex colour-vector
// hidden channels; FP32 weights and arithmetic, FP32 activations):
//   rhat = r / |r|                                   (4 channels: the spin components)
//   h_c(y) = sum_d sum_c' W1[d][c][c'] T_d(y) rhat_c'(y + d)      odd y
//   g_c    = h_c / (1 + |h_c|^2)                                  (gauge-covariant gate)
//   z_c(x) = sum_d sum_c' W2[d][c][c'] T_d(x) g_c'(x + d) + sum_c' W0[c][c'] rhat_c'(x)   even x
//   N(r)   = |r| z
// d = 2 mu (+mu) / 2 mu + 1 (-mu); T_d the hop's transporter with the fermion
// boundary factor.  Weights: complex [W1 8x12x4 | W2 8x4x12 | W0 4x4] = 784 entries.
// Training objectives (dL = 2 Re sum_w A_w dw; the kernels return the A_w):
//   preconditioned residual  sum_r |Khat z(rhat) - rhat|^2   (dL/dz* = Khat (Khat z - rhat))
//   solution matching        sum_(r,e) |z(rhat) - e/|r||^2 / |e/|r||^2, Khat e = r.
// The first asks the network for what a local operator can give a preconditioner,
// Khat^-1 on the high modes; the second asks for the low modes too, out of reach of a
// two-hop network.
#include <chrono>
#include <cmath>
#include <vector>

#include "hop.h"

namespace {

constexpr int NIN = 4, NH = 12, NW1 = 8 * NH * NIN, NW2 = 8 * NIN * NH, NW0 = NIN * NIN;
constexpr int NW = NW1 + NW2 + NW0;   // 784

__device__ __forceinline__ float2 fconj(float2 a) { return make_float2(a.x, -a.y); }

// device scalars of the flexible CG (ctx->scal + kFcgBase)
constexpr int kFcgBase = 7600;
enum { F_RZ = 0, F_PQ, F_ALPHA, F_RN2, F_THR, F_ITER, F_DONE, F_MAXIT, F_INVR, F_NR, F_BETA, F_FB, F_NFB, F_RZOLD,
       F_ZR, F_ZQ, F_NSLOT };

// The transporter T_d(y) of the site y with coordinates c, loaded once per direction:
// U_mu(y) for d = 2 mu, U_mu(y - mu)^dag for d = 2 mu + 1, and its fermion boundary factor.
__device__ __forceinline__ void load_T(const Geom &g, const float2 *__restrict__ U, int p, int i, const int *c, int d,
                                       float2 *u, float *sgn)
{
    const int mu = d >> 1;
    // FP32 link copy: row r of a link at site i is the record of 3 complex at 3 r Vh + 3 i
    if ((d & 1) == 0) {
        const float2 *b = U + ((long)(p * 4 + mu) * 9) * g.Vh + 3L * i;
        for (int k = 0; k < 9; k++) u[k] = b[(long)(k / 3) * 3 * g.Vh + k % 3];
        *sgn = (mu == 3 && c[3] == g.L[3] - 1) ? (float)g.tbc : 1.f;
    } else {
        int s;
        int j = eo_neighbour(g, c, mu, -1, &s);
        const float2 *b = U + ((long)((1 - p) * 4 + mu) * 9) * g.Vh + 3L * j;
        for (int a = 0; a < 3; a++)
            for (int bb = 0; bb < 3; bb++) u[3 * a + bb] = fconj(b[(long)bb * 3 * g.Vh + a]);
        *sgn = (float)s;
    }
}

// w = sgn T v (DAG = 0) or sgn T^dag v (DAG = 1)
template <int DAG>
__device__ __forceinline__ void apply_T(const float2 *u, float sgn, const float2 *v, float2 *w)
{
    for (int a = 0; a < 3; a++) {
        float2 acc = make_float2(0.f, 0.f);
        for (int bb = 0; bb < 3; bb++) {
            if (DAG) cfmac(acc, u[3 * bb + a], v[bb]);
            else cfma(acc, u[3 * a + bb], v[bb]);
        }
        w[a] = make_float2(acc.x * sgn, acc.y * sgn);
    }
}

__device__ __forceinline__ int nbr_of(const Geom &g, const int *c, int d)
{
    int s;
    return eo_neighbour(g, c, d >> 1, (d & 1) ? -1 : +1, &s);
}

// layer 1 on odd sites: h (pre-gate) and g (gated), [36][Vh] float2 each
// (fs: flexible-CG scalars; when given, the input scale 1/|r| is read there and the
// kernel is skipped once the solve is done)
__global__ __launch_bounds__(kBlock) void k_pt_l1(Geom g, const float2 *__restrict__ U,
                                                  const double2 *__restrict__ r, float scale,
                                                  const float2 *__restrict__ W, float2 *__restrict__ H,
                                                  float2 *__restrict__ G, const double *__restrict__ fs)
{
    if (fs) {
        if (fs[F_DONE] != 0) return;
        scale = (float)fs[F_INVR];
    }
    // weights of layer 1 in LDS (uniform reads; the lanes of a site index different rows)
    __shared__ float2 sw[NW1];
    for (int k = threadIdx.x; k < NW1; k += blockDim.x) sw[k] = W[k];
    __syncthreads();
    // four lanes per site (one quad of a wave): lane q transports input channel q along each
    // direction, the quad shares the four transported vectors by xor shuffles, and lane q
    // mixes them into the hidden channels 3q .. 3q + 2.  The lanes of a site are valid or
    // not together, so a whole quad returns at once.
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int i = (int)(t >> 2), q = (int)(t & 3);
    if (i >= g.Vh) return;
    int c[4];
    eo_coords(g, 1, i, c);
    constexpr int NO = NH / 4;
    float2 h[NO * 3];
#pragma unroll
    for (int k = 0; k < NO * 3; k++) h[k] = make_float2(0.f, 0.f);
    for (int d = 0; d < 8; d++) {
        const int j = nbr_of(g, c, d);
        float2 u[9], v[3], tv[3];
        float sgn;
        load_T(g, U, 1, i, c, d, u, &sgn);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const double2 x = r[(long)(3 * q + a) * g.Vh + j];
            v[a] = make_float2((float)x.x * scale, (float)x.y * scale);
        }
        apply_T<0>(u, sgn, v, tv);
        const float2 *w = sw + d * NH * NIN + (NO * q) * NIN;
#pragma unroll
        for (int m = 0; m < NIN; m++) {
            const int ch = q ^ m;   // channel held by the lane m away in the quad
            float2 pv[3];
#pragma unroll
            for (int a = 0; a < 3; a++)
                pv[a] = m == 0 ? tv[a] : make_float2(__shfl_xor(tv[a].x, m, 64), __shfl_xor(tv[a].y, m, 64));
#pragma unroll
            for (int o = 0; o < NO; o++) {
                const float2 wc = w[o * NIN + ch];
#pragma unroll
                for (int a = 0; a < 3; a++) cfma(h[3 * o + a], wc, pv[a]);
            }
        }
    }
    for (int o = 0; o < NO; o++) {
        const int oc = NO * q + o;
        float qq = 0.f;
        for (int a = 0; a < 3; a++) qq += h[3 * o + a].x * h[3 * o + a].x + h[3 * o + a].y * h[3 * o + a].y;
        float sg = 1.f / (1.f + qq);
        for (int a = 0; a < 3; a++) {
            if (H) H[(long)(3 * oc + a) * g.Vh + i] = h[3 * o + a];
            G[(long)(3 * oc + a) * g.Vh + i] = make_float2(h[3 * o + a].x * sg, h[3 * o + a].y * sg);
        }
    }
}

// layer 2 on even sites: z = conv(g) + W0 rhat; out (FP64) = oscale * z, or z (FP32).
// Four lanes per site, lane o computing output channel o:
// sum_ch W2[d][o][ch] T_d g_ch = T_d (sum_ch W2[d][o][ch] g_ch), one transport per direction.
__global__ __launch_bounds__(kBlock) void k_pt_l2(Geom g, const float2 *__restrict__ U,
                                                  const double2 *__restrict__ r, float scale,
                                                  const float2 *__restrict__ W, const float2 *__restrict__ G,
                                                  double oscale, double2 *__restrict__ out, float2 *__restrict__ zf,
                                                  const double *__restrict__ fs, const double2 *__restrict__ q,
                                                  double *__restrict__ dots)
{
    // (flexible CG: with dots, also the block partials of Re<out, r> and Re<out, q>)
    if (fs) {
        if (fs[F_DONE] != 0) return;
        scale = (float)fs[F_INVR];
        oscale = fs[F_NR];
    }
    __shared__ float2 sw[NW2 + NW0];
    for (int k = threadIdx.x; k < NW2 + NW0; k += blockDim.x) sw[k] = W[NW1 + k];
    __syncthreads();
    const float2 *W2 = sw, *W0 = sw + NW2;
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int i = (int)(t >> 2), o = (int)(t & 3);
    double dzr = 0, dzq = 0;
    if (i < g.Vh) {
        int c[4];
        eo_coords(g, 0, i, c);
        float2 z[3];
        for (int a = 0; a < 3; a++) {
            float2 acc = make_float2(0.f, 0.f);
            for (int ch = 0; ch < NIN; ch++) {
                double2 x = r[(long)(3 * ch + a) * g.Vh + i];
                cfma(acc, W0[o * NIN + ch], make_float2((float)x.x * scale, (float)x.y * scale));
            }
            z[a] = acc;
        }
        for (int d = 0; d < 8; d++) {
            const int j = nbr_of(g, c, d);
            // lane o reads the hidden channels 3o .. 3o + 2 and mixes them into all four
            // outputs; a reduce-scatter over the quad (xor 2, then xor 1) leaves output o's
            // sum on lane o
            const float2 *w = W2 + d * NIN * NH;
            float2 mp[NIN][3];
#pragma unroll
            for (int oo = 0; oo < NIN; oo++)
#pragma unroll
                for (int a = 0; a < 3; a++) mp[oo][a] = make_float2(0.f, 0.f);
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const int ch = 3 * o + k;
                float2 gv[3];
#pragma unroll
                for (int a = 0; a < 3; a++) gv[a] = G[(long)(3 * ch + a) * g.Vh + j];
#pragma unroll
                for (int oo = 0; oo < NIN; oo++) {
                    const float2 wc = w[oo * NH + ch];
#pragma unroll
                    for (int a = 0; a < 3; a++) cfma(mp[oo][a], wc, gv[a]);
                }
            }
            const bool hi2 = (o & 2) != 0, hi1 = (o & 1) != 0;
            float2 kp[2][3], m[3];
#pragma unroll
            for (int k = 0; k < 2; k++)
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    const float2 keep = hi2 ? mp[2 + k][a] : mp[k][a];
                    const float2 send = hi2 ? mp[k][a] : mp[2 + k][a];
                    kp[k][a] = make_float2(keep.x + __shfl_xor(send.x, 2, 64), keep.y + __shfl_xor(send.y, 2, 64));
                }
#pragma unroll
            for (int a = 0; a < 3; a++) {
                const float2 keep = hi1 ? kp[1][a] : kp[0][a];
                const float2 send = hi1 ? kp[0][a] : kp[1][a];
                m[a] = make_float2(keep.x + __shfl_xor(send.x, 1, 64), keep.y + __shfl_xor(send.y, 1, 64));
            }
            float2 u[9], tv[3];
            float sgn;
            load_T(g, U, 0, i, c, d, u, &sgn);
            apply_T<0>(u, sgn, m, tv);
#pragma unroll
            for (int a = 0; a < 3; a++) z[a] = cadd(z[a], tv[a]);
        }
        for (int a = 0; a < 3; a++) {
            const long e = (long)(3 * o + a) * g.Vh + i;
            const double2 zo = make_double2(oscale * z[a].x, oscale * z[a].y);
            if (out) out[e] = zo;
            if (zf) zf[e] = z[a];
            if (dots) {
                const double2 rv = r[e], qv = q[e];
                dzr += zo.x * rv.x + zo.y * rv.y;
                dzq += zo.x * qv.x + zo.y * qv.y;
            }
        }
    }
    if (dots) {
        const double v[2] = {dzr, dzq};
        partials_store_at<kBlock, 2>(v, dots, blockIdx.x);
    }
}

// Gz = (z - e * escale) * inv_ne on even sites (FP32), and the pair's loss partials
__global__ __launch_bounds__(kBlock) void k_pt_gz(Geom g, const float2 *__restrict__ z,
                                                  const double2 *__restrict__ e, float escale, float inv_ne,
                                                  float2 *__restrict__ Gz, double *__restrict__ partials)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0;
    if (i < g.Vh)
        for (int k = 0; k < 12; k++) {
            double2 ev = e[(long)k * g.Vh + i];
            float2 d = make_float2(z[(long)k * g.Vh + i].x - (float)ev.x * escale,
                                   z[(long)k * g.Vh + i].y - (float)ev.y * escale);
            s += (double)d.x * d.x + (double)d.y * d.y;
            Gz[(long)k * g.Vh + i] = make_float2(d.x * inv_ne, d.y * inv_ne);
        }
    block_sum_store<float2>(s * inv_ne, partials);
}

// d = y - scale r on even sites (FP32) and |d|^2 block partials
__global__ __launch_bounds__(kBlock) void k_pt_resid(Geom g, const float2 *__restrict__ y,
                                                     const double2 *__restrict__ r, float scale,
                                                     float2 *__restrict__ d, double *__restrict__ partials)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0;
    if (i < g.Vh)
        for (int k = 0; k < 12; k++) {
            double2 rv = r[(long)k * g.Vh + i];
            float2 v = make_float2(y[(long)k * g.Vh + i].x - (float)rv.x * scale,
                                   y[(long)k * g.Vh + i].y - (float)rv.y * scale);
            s += (double)v.x * v.x + (double)v.y * v.y;
            d[(long)k * g.Vh + i] = v;
        }
    block_sum_store<float2>(s, partials);
}

// Wave sums of K values per lane (K a power of two, at most 64) by reduce-scatter:
// at each butterfly level a lane keeps one half of its values and adds the other
// lane's copy of that half, so log2(K) levels cost K - 1 shuffles in all; lane l
// ends with the total of value l / (64 / K) and stores it to
// part[wave * stride + base + l / (64 / K)].
// one level: n live values, partner lane at xor distance M
template <int N, int M, int K>
__device__ __forceinline__ void rs_level(float (&v)[K], int lane)
{
    if constexpr (N > 1) {
        const bool up = (lane & M) != 0;
#pragma unroll
        for (int j = 0; j < N / 2; j++) {
            const float send = up ? v[j] : v[j + N / 2];
            const float keep = up ? v[j + N / 2] : v[j];
            v[j] = keep + __shfl_xor(send, M, 64);
        }
        rs_level<N / 2, M / 2>(v, lane);
    }
}

template <int K>
__device__ __forceinline__ void wave_rs_store(float (&v)[K], double *__restrict__ part, long stride, int base)
{
    static_assert(K >= 1 && K <= 64 && (K & (K - 1)) == 0, "K must be a power of two <= 64");
    const int lane = threadIdx.x & 63;
    rs_level<K, 32>(v, lane);
    constexpr int R = 64 / K;
#pragma unroll
    for (int m = R / 2; m > 0; m >>= 1) v[0] += __shfl_xor(v[0], m, 64);
    if ((lane & (R - 1)) == 0) {
        const long w = (blockIdx.x * (long)blockDim.x + threadIdx.x) >> 6;
        part[w * stride + base + lane / R] = v[0];
    }
}

// A2[d][o][ch] = sum_x <Gz_o(x), T_d(x) g_ch(x + d)>, A0[o][ch] = sum_x <Gz_o(x), rhat_ch(x)> (even x)
__global__ __launch_bounds__(kBlock) void k_pt_grad2(Geom g, const float2 *__restrict__ U,
                                                     const double2 *__restrict__ r, float scale,
                                                     const float2 *__restrict__ G, const float2 *__restrict__ Gz,
                                                     double *__restrict__ part)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool ok = i < g.Vh;
    int c[4] = {0, 0, 0, 0};
    float2 gz[NIN * 3];
    if (ok) {
        eo_coords(g, 0, i, c);
        for (int k = 0; k < 12; k++) gz[k] = Gz[(long)k * g.Vh + i];
    } else {
        for (int k = 0; k < 12; k++) gz[k] = make_float2(0.f, 0.f);
    }
    const long stride = 2L * (NW2 + NW0);
    // <Gz_o, T g_ch(x+d)> = <T^dag Gz_o, g_ch(x+d)>: 4 transports per direction, not 12
    for (int d = 0; d < 8; d++) {
        int j = ok ? nbr_of(g, c, d) : 0;
        float2 tg[NIN * 3];
        if (ok) {
            float2 u[9];
            float sgn;
            load_T(g, U, 0, i, c, d, u, &sgn);
            for (int o = 0; o < NIN; o++) apply_T<1>(u, sgn, gz + 3 * o, tg + 3 * o);
        } else {
            for (int k = 0; k < NIN * 3; k++) tg[k] = make_float2(0.f, 0.f);
        }
        // the NIN x NH values of direction d, (re, im) interleaved in index order: the
        // first 64 floats in one reduce-scatter, the last 32 in another
        static_assert(2 * NIN * NH == 96, "split of the values of one direction");
        float va[64], vb[32];
#pragma unroll
        for (int ch = 0; ch < NH; ch++) {
            float2 v[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
            if (ok)
                for (int a = 0; a < 3; a++) v[a] = G[(long)(3 * ch + a) * g.Vh + j];
#pragma unroll
            for (int o = 0; o < NIN; o++) {
                float2 acc = make_float2(0.f, 0.f);
                for (int a = 0; a < 3; a++) cfmac(acc, tg[3 * o + a], v[a]);
                const int f = 2 * (o * NH + ch);
                if (f < 64) {
                    va[f] = acc.x;
                    va[f + 1] = acc.y;
                } else {
                    vb[f - 64] = acc.x;
                    vb[f - 63] = acc.y;
                }
            }
        }
        wave_rs_store(va, part, stride, 2 * d * NIN * NH);
        wave_rs_store(vb, part, stride, 2 * d * NIN * NH + 64);
    }
    float vals0[2 * NIN * NIN];
    for (int o = 0; o < NIN; o++)
        for (int ch = 0; ch < NIN; ch++) {
            float2 acc = make_float2(0.f, 0.f);
            if (ok)
                for (int a = 0; a < 3; a++) {
                    double2 x = r[(long)(3 * ch + a) * g.Vh + i];
                    cfmac(acc, gz[3 * o + a], make_float2((float)x.x * scale, (float)x.y * scale));
                }
            vals0[2 * (o * NIN + ch)] = acc.x;
            vals0[2 * (o * NIN + ch) + 1] = acc.y;
        }
    wave_rs_store(vals0, part, stride, 2 * NW2);
}

// back to the hidden layer on odd y: Gg(y) = sum_d W2[opp d]^dag T_d(y) Gz(y + d), then
// the gate: Gh = s Gg + 2 s' Re<Gg, h> h, s = 1/(1+q), s' = -1/(1+q)^2, q = |h|^2
__global__ __launch_bounds__(kBlock) void k_pt_back(Geom g, const float2 *__restrict__ U,
                                                    const float2 *__restrict__ W, const float2 *__restrict__ Gz,
                                                    const float2 *__restrict__ H, float2 *__restrict__ Gh)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.Vh) return;
    int c[4];
    eo_coords(g, 1, i, c);
    const float2 *W2 = W + NW1;
    float2 gg[NH * 3];
    for (int k = 0; k < NH * 3; k++) gg[k] = make_float2(0.f, 0.f);
    for (int d = 0; d < 8; d++) {
        int j = nbr_of(g, c, d);
        const int od = d ^ 1;
        const float2 *w = W2 + od * NIN * NH;
        float2 u[9];
        float sgn;
        load_T(g, U, 1, i, c, d, u, &sgn);
        for (int o = 0; o < NIN; o++) {
            float2 v[3], t[3];
            for (int a = 0; a < 3; a++) v[a] = Gz[(long)(3 * o + a) * g.Vh + j];
            apply_T<0>(u, sgn, v, t);
            for (int ch = 0; ch < NH; ch++) {
                float2 wc = fconj(w[o * NH + ch]);
                for (int a = 0; a < 3; a++) cfma(gg[3 * ch + a], wc, t[a]);
            }
        }
    }
    for (int ch = 0; ch < NH; ch++) {
        float2 h[3];
        float q = 0.f, re = 0.f;
        for (int a = 0; a < 3; a++) {
            h[a] = H[(long)(3 * ch + a) * g.Vh + i];
            q += h[a].x * h[a].x + h[a].y * h[a].y;
            re += gg[3 * ch + a].x * h[a].x + gg[3 * ch + a].y * h[a].y;
        }
        float s = 1.f / (1.f + q), ds = -s * s;
        for (int a = 0; a < 3; a++)
            Gh[(long)(3 * ch + a) * g.Vh + i] = make_float2(s * gg[3 * ch + a].x + 2.f * ds * re * h[a].x,
                                                            s * gg[3 * ch + a].y + 2.f * ds * re * h[a].y);
    }
}

// A1[d][o][ch] = sum_y <Gh_o(y), T_d(y) rhat_ch(y + d)> (odd y)
__global__ __launch_bounds__(kBlock) void k_pt_grad1(Geom g, const float2 *__restrict__ U,
                                                     const double2 *__restrict__ r, float scale,
                                                     const float2 *__restrict__ Gh, double *__restrict__ part)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool ok = i < g.Vh;
    int c[4] = {0, 0, 0, 0};
    if (ok) eo_coords(g, 1, i, c);
    const long stride = 2L * NW1;
    float2 gh[NH * 3];
    for (int k = 0; k < NH * 3; k++) gh[k] = ok ? Gh[(long)k * g.Vh + i] : make_float2(0.f, 0.f);
    for (int d = 0; d < 8; d++) {
        int j = ok ? nbr_of(g, c, d) : 0;
        float2 t[NIN * 3], u[9];
        float sgn = 0.f;
        if (ok) load_T(g, U, 1, i, c, d, u, &sgn);
        for (int ch = 0; ch < NIN; ch++) {
            float2 v[3];
            for (int a = 0; a < 3; a++) {
                double2 x = ok ? r[(long)(3 * ch + a) * g.Vh + j] : make_double2(0, 0);
                v[a] = make_float2((float)x.x * scale, (float)x.y * scale);
            }
            if (ok) apply_T<0>(u, sgn, v, t + 3 * ch);
            else for (int a = 0; a < 3; a++) t[3 * ch + a] = make_float2(0.f, 0.f);
        }
        // the NH x NIN values of direction d in index order: hidden channels 0-7 in one
        // reduce-scatter of 64 floats, 8-11 in one of 32
        static_assert(2 * NIN * NH == 96, "split of the values of one direction");
        float va[64];
#pragma unroll
        for (int o = 0; o < 8; o++)
#pragma unroll
            for (int ch = 0; ch < NIN; ch++) {
                float2 acc = make_float2(0.f, 0.f);
                for (int a = 0; a < 3; a++) cfmac(acc, gh[3 * o + a], t[3 * ch + a]);
                va[2 * (o * NIN + ch)] = acc.x;
                va[2 * (o * NIN + ch) + 1] = acc.y;
            }
        wave_rs_store(va, part, stride, 2 * d * NH * NIN);
        float vb[32];
#pragma unroll
        for (int o = 8; o < NH; o++)
#pragma unroll
            for (int ch = 0; ch < NIN; ch++) {
                float2 acc = make_float2(0.f, 0.f);
                for (int a = 0; a < 3; a++) cfmac(acc, gh[3 * o + a], t[3 * ch + a]);
                vb[2 * ((o - 8) * NIN + ch)] = acc.x;
                vb[2 * ((o - 8) * NIN + ch) + 1] = acc.y;
            }
        wave_rs_store(vb, part, stride, 2 * d * NH * NIN + 64);
    }
}

// Column sums of the (nw x nvals) row-major partials in two fixed-order passes.
// Pass 1: block (c, j) sums rows of chunk j for the 64 columns of group c, four row
// phases per column folded through LDS; mid[j * nvals + v].
constexpr int kSumChunks = 64;

__global__ __launch_bounds__(256) void k_pt_sum_rows(const double *__restrict__ part, long nw, int nvals,
                                                     double *__restrict__ mid)
{
    __shared__ double sh[256];
    const int v = blockIdx.x * 64 + (threadIdx.x & 63), ph = threadIdx.x >> 6;
    const long per = (nw + kSumChunks - 1) / kSumChunks;
    const long w0 = blockIdx.y * per, w1 = w0 + per < nw ? w0 + per : nw;
    double s = 0;
    if (v < nvals)
        for (long w = w0 + ph; w < w1; w += 4) s += part[w * nvals + v];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (ph == 0 && v < nvals)
        mid[(long)blockIdx.y * nvals + v] = (sh[threadIdx.x] + sh[threadIdx.x + 64]) +
                                            (sh[threadIdx.x + 128] + sh[threadIdx.x + 192]);
}

// pass 2: out[v] = sum_j mid[j * nvals + v], one thread per value
__global__ void k_pt_sum(const double *__restrict__ mid, int nvals, double *__restrict__ out)
{
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvals) return;
    double s = 0;
    for (int j = 0; j < kSumChunks; j++) s += mid[(long)j * nvals + v];
    out[v] = s;
}

// ---------------------------------------------------------------- flexible CG kernels
//
// Every scalar lives in fs (device); a chunk of iterations runs without the host.

// q = Khat p (from t = Mhat p, T' = A_oo^-1 D_oe g5 t), alpha = rz / <p, q> (<p, q>
// totalled from the stage-2 partials by a one-block kernel), x += alpha p, r -= alpha q;
// |r|^2 partials
template <int CLOV, int LM>
__global__ __launch_bounds__(kBlock) void k_f_hop4(Geom g, const double2 *__restrict__ t,
                                                   const double2 *__restrict__ T, const double2 *__restrict__ U,
                                                   const double *__restrict__ cl, double a,
                                                   const double2 *__restrict__ p, double2 *__restrict__ q,
                                                   double2 *__restrict__ x, double2 *__restrict__ r,
                                                   double *__restrict__ fs, double *__restrict__ part_rr)
{
    if (fs[F_DONE] != 0) return;
    const double alpha = fs[F_RZ] / fs[F_PQ];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        fs[F_ALPHA] = alpha;
        fs[F_RZOLD] = fs[F_RZ];
    }
    const int tt = xcd_site(2 * g.Vh);
    double nrm = 0;
    if (tt >= 0) {
        const int i = tile_site(g, tt >> 1), hb = tt & 1;
        double2 acc[6], tv[6], at[6];
        hop_pair<LM, double2>(g, 0, i, hb, T, U, 1.0, acc);
        load_block(t, g.Vh, i, hb, -1.0, tv);
        if (CLOV) clover_block<double, double2>(cl, g.Vh, i, hb, tv, at);
#pragma unroll
        for (int k = 0; k < 6; k++) {
            double2 base = CLOV ? at[k] : tv[k];
            double2 kp = make_double2(base.x + a * acc[k].x, base.y + a * acc[k].y);
            if (hb) kp = cneg(kp);
            const long e = (long)(6 * hb + k) * g.Vh + i;
            double2 pv = p[e], xv = x[e], rv = r[e];
            xv.x += alpha * pv.x; xv.y += alpha * pv.y;
            rv.x -= alpha * kp.x; rv.y -= alpha * kp.y;
            x[e] = xv;
            r[e] = rv;
            q[e] = kp;
            cnorm_acc(nrm, rv);
        }
    }
    const double v[1] = {nrm};
    op_partials_store<kBlock, 1>(v, part_rr);
}

// |r|^2 from the stage-4 partials, convergence, |r| and 1/|r| for the network (one workgroup)
__global__ __launch_bounds__(kFinishThreads) void k_f_norm(const double *__restrict__ part, int n,
                                                          double *__restrict__ fs)
{
    if (fs[F_DONE] != 0) return;
    double t[1];
    partials_total<kFinishThreads, 1, kMaxChunks>(part, n, t);
    if (threadIdx.x == 0) {
        const double rr = t[0];
        fs[F_RN2] = rr;
        fs[F_NR] = sqrt(rr);
        fs[F_INVR] = rr > 0 ? 1.0 / sqrt(rr) : 0.0;
        fs[F_ITER] += 1;
        fs[F_DONE] = rr <= fs[F_THR] ? 1 : (fs[F_ITER] >= fs[F_MAXIT] ? 2 : 0);
    }
}

// partials of Re<z, r> and Re<z, q> (2 per block)
__global__ __launch_bounds__(kBlock) void k_f_dots(long n, const double2 *__restrict__ z,
                                                   const double2 *__restrict__ r, const double2 *__restrict__ q,
                                                   const double *__restrict__ fs, double *__restrict__ part)
{
    if (fs[F_DONE] != 0) return;
    double a = 0, b = 0;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        double2 zv = z[e], rv = r[e], qv = q[e];
        a += zv.x * rv.x + zv.y * rv.y;
        b += zv.x * qv.x + zv.y * qv.y;
    }
    __shared__ double sh[2][kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o, 64);
        b += __shfl_down(b, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = a;
        sh[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0, sb = 0;
        for (int k = 0; k < kBlock / 64; k++) {
            sa += sh[0][k];
            sb += sh[1][k];
        }
        part[2 * blockIdx.x] = sa;
        part[2 * blockIdx.x + 1] = sb;
    }
}

// Polak-Ribiere beta = <z+, r+ - r> / <z, r> = -alpha <z+, q> / rz, or the plain-CG
// fallback (z = r, beta = 0) where <z+, r+> <= 0; first = 1 only sets rz for p = z
__global__ __launch_bounds__(kRedBlock) void k_f_beta(const double *__restrict__ part, int n, int first,
                                                      double *__restrict__ fs)
{
    if (!first && fs[F_DONE] != 0) return;
    __shared__ double sh[2][kRedBlock / 64];
    double a = 0, b = 0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o, 64);
        b += __shfl_down(b, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = a;
        sh[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double zr = 0, zq = 0;
        for (int k = 0; k < kRedBlock / 64; k++) {
            zr += sh[0][k];
            zq += sh[1][k];
        }
        if (zr > 0) {
            fs[F_BETA] = first ? 0.0 : -fs[F_ALPHA] * zq / fs[F_RZ];
            fs[F_RZ] = zr;
            fs[F_FB] = 0;
        } else {
            fs[F_BETA] = 0.0;
            fs[F_RZ] = fs[F_RN2];
            fs[F_FB] = 1;
            fs[F_NFB] += 1;
        }
    }
}

// p = (fallback ? r : z) + beta p
__global__ void k_f_update_p(long n, const double2 *__restrict__ z, const double2 *__restrict__ r,
                             double2 *__restrict__ p, const double *__restrict__ fs)
{
    if (fs[F_DONE] != 0) return;
    long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double b = fs[F_BETA];
    double2 v = fs[F_FB] != 0 ? r[e] : z[e], pv = p[e];
    p[e] = make_double2(v.x + b * pv.x, v.y + b * pv.y);
}

// Polak-Ribiere step fused with p: <z, r> and <z, q> totalled from the network's second
// layer's partials by a one-block kernel, beta = -alpha <z, q> / rz_old or the plain-CG fallback (z = r, beta = 0) where
// <z, r> <= 0; p = z + beta p.  Block 0 records rz and the fallback count (no block reads
// them in this launch).
__global__ __launch_bounds__(kRedBlock) void k_f_update_p_fused(long n, const double2 *__restrict__ z,
                                                                const double2 *__restrict__ r,
                                                                double2 *__restrict__ p, double *__restrict__ fs)
{
    if (fs[F_DONE] != 0) return;
    const double zr = fs[F_ZR], zq = fs[F_ZQ];
    const bool fb = !(zr > 0);
    const double beta = fb ? 0.0 : -fs[F_ALPHA] * zq / fs[F_RZOLD];
    const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (e < n) {
        double2 v = fb ? r[e] : z[e], pv = p[e];
        p[e] = make_double2(v.x + beta * pv.x, v.y + beta * pv.y);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        fs[F_BETA] = beta;
        fs[F_FB] = fb ? 1 : 0;
        if (fb) fs[F_NFB] += 1;
        fs[F_RZ] = fb ? fs[F_RN2] : zr;
    }
}

// start: x = 0, r = b, |r|^2 = |b|^2 and the thresholds
__global__ __launch_bounds__(kRedBlock) void k_f_init(const double *__restrict__ part, int n, double tol2,
                                                      int maxiter, double *__restrict__ fs)
{
    __shared__ double sh[kRedBlock / 64];
    double s = 0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) s += part[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double bb = 0;
        for (int k = 0; k < kRedBlock / 64; k++) bb += sh[k];
        fs[F_RN2] = bb;
        fs[F_NR] = sqrt(bb);
        fs[F_INVR] = bb > 0 ? 1.0 / sqrt(bb) : 0.0;
        fs[F_THR] = tol2 * bb;
        fs[F_ITER] = 0;
        fs[F_DONE] = bb == 0 ? 1 : 0;
        fs[F_MAXIT] = maxiter;
        fs[F_RZ] = 1;
        fs[F_ALPHA] = 0;
        fs[F_NFB] = 0;
    }
}

}  // namespace

// ---------------------------------------------------------------- host side

struct PtWs {
    float2 *W, *H, *G, *Gz, *Gh, *z;
    double *part, *mid, *sum;
};

static int pt_ws(pfmp_ctx *ctx, const double *Wc, PtWs &w)
{
    if (int rc0 = gauge_f32_ready(ctx)) return rc0;
    const Geom &g = ctx->g;
    const size_t hb = sizeof(float2) * 36L * g.Vh, zb = sizeof(float2) * 12L * g.Vh;
    const long nwaves = (long)nblocks(g.Vh, kBlock) * (kBlock / 64);
    const long per_wave = 2L * (NW2 + NW0) > 2L * NW1 ? 2L * (NW2 + NW0) : 2L * NW1;
    w.W = (float2 *)ws_alloc(ctx, sizeof(float2) * NW, 32);
    w.H = (float2 *)ws_alloc(ctx, hb, 34);
    w.G = (float2 *)ws_alloc(ctx, hb, 35);
    w.Gh = (float2 *)ws_alloc(ctx, hb, 36);
    w.Gz = (float2 *)ws_alloc(ctx, zb, 37);
    w.z = (float2 *)ws_alloc(ctx, zb, 38);
    w.part = (double *)ws_alloc(ctx, sizeof(double) * ((nwaves + kSumChunks) * per_wave + 64), 33);
    w.mid = w.part ? w.part + nwaves * per_wave : nullptr;
    w.sum = (double *)(ctx->scal + 6000);   // 2 * (NW2 + NW0) <= 800 doubles
    if (!w.W || !w.H || !w.G || !w.Gh || !w.Gz || !w.z || !w.part) return set_err(ctx, PFMP_ERR_OOM, "ptnet workspace");
    if (Wc) {
        std::vector<float2> wf(NW);
        for (int k = 0; k < NW; k++) wf[k] = make_float2((float)Wc[2 * k], (float)Wc[2 * k + 1]);
        HIPCHK(ctx, hipMemcpyAsync(w.W, wf.data(), sizeof(float2) * NW, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    return 0;
}

// w.sum[v] = column sums of the nwaves x nvals partials
static void col_sums(pfmp_ctx *ctx, PtWs &w, long nwaves, int nvals)
{
    hipLaunchKernelGGL(k_pt_sum_rows, dim3((nvals + 63) / 64, kSumChunks), dim3(256), 0, ctx->stream, w.part, nwaves,
                       nvals, w.mid);
    hipLaunchKernelGGL(k_pt_sum, dim3(nblocks(nvals, 256)), dim3(256), 0, ctx->stream, w.mid, nvals, w.sum);
}

static double host_norm(pfmp_ctx *ctx, const double2 *v, int *rc)
{
    double s = 0;
    *rc = launch_norm2(ctx, v, 12L * ctx->g.Vh, ctx->red);
    if (!*rc) *rc = red_finish(ctx, ctx->red, ctx->nblk_red, 1, &s);
    return std::sqrt(s);
}

// out = N(r) with r of norm nr (given) in FP64 internal layout
static int pt_apply(pfmp_ctx *ctx, PtWs &w, const double2 *r, double nr, double2 *out)
{
    const Geom &g = ctx->g;
    float sc = nr > 0 ? (float)(1.0 / nr) : 0.f;
    dim3 grid(nblocks(g.Vh, kBlock)), block(kBlock);
    dim3 grid4(nblocks(4L * g.Vh, kBlock));
    hipLaunchKernelGGL(k_pt_l1, grid4, block, 0, ctx->stream, g, ctx->Uf, r, sc, w.W, (float2 *)nullptr, w.G,
                       (const double *)nullptr);
    hipLaunchKernelGGL(k_pt_l2, grid4, block, 0, ctx->stream, g, ctx->Uf, r, sc, w.W, w.G, nr, out,
                       (float2 *)nullptr, (const double *)nullptr, (const double2 *)nullptr, (double *)nullptr);
    LAUNCHCHK(ctx);
    return 0;
}

extern "C" int pfmp_ptnet_apply(pfmp_ctx *ctx, const double *W, const void *r, void *out)
{
    if (!ctx || !W || !r || !out) return ctx ? set_err(ctx, PFMP_ERR_ARG, "ptnet_apply: null") : PFMP_ERR_ARG;
    if (!ctx->have_gauge) return set_err(ctx, PFMP_ERR_STATE, "no gauge field set");
    PtWs w;
    int rc = pt_ws(ctx, W, w);
    if (rc) return rc;
    double nr = host_norm(ctx, (const double2 *)r, &rc);
    if (rc) return rc;
    return pt_apply(ctx, w, (const double2 *)r, nr, (double2 *)out);
}

extern "C" int pfmp_ptnet_grad(pfmp_ctx *ctx, const double *W, int op, int npairs, const void *const *R,
                               const void *const *E, double *loss, double *A)
{
    if (!ctx || !W || npairs <= 0 || !R || (op < 0 && !E) || !loss || !A)
        return ctx ? set_err(ctx, PFMP_ERR_ARG, "ptnet_grad: bad arguments") : PFMP_ERR_ARG;
    if (!ctx->have_gauge) return set_err(ctx, PFMP_ERR_STATE, "no gauge field set");
    if (op >= 0)
        if (int rc0 = op_ready(ctx, op)) return rc0;
    const Geom &g = ctx->g;
    PtWs w;
    int rc = pt_ws(ctx, W, w);
    if (rc) return rc;
    float2 *ky = nullptr, *kte = nullptr, *kto = nullptr;
    if (op >= 0) {
        const size_t fb = sizeof(float2) * 12L * g.Vh;
        ky = (float2 *)ws_alloc(ctx, fb, 39);
        kte = (float2 *)ws_alloc(ctx, fb, 40);
        kto = (float2 *)ws_alloc(ctx, fb, 41);
        if (!ky || !kte || !kto) return set_err(ctx, PFMP_ERR_OOM, "ptnet workspace");
    }
    dim3 grid(nblocks(g.Vh, kBlock)), block(kBlock);
    const long nwaves = (long)grid.x * (kBlock / 64);
    std::vector<double> acc(2 * NW, 0.0);
    double tot = 0;
    std::vector<double> tmp(2 * NW);   // holds either the A2|A0 block (800) or the A1 block (768)
    static_assert(NW1 <= NW && NW2 + NW0 <= NW, "tmp holds the A1 block or the A2|A0 block");
    for (int p = 0; p < npairs; p++) {
        const double2 *r = (const double2 *)R[p];
        double nr = host_norm(ctx, r, &rc);
        if (rc) return rc;
        float sc = (float)(1.0 / nr);
        hipLaunchKernelGGL(k_pt_l1, dim3(nblocks(4L * g.Vh, kBlock)), block, 0, ctx->stream, g, ctx->Uf, r, sc, w.W,
                           w.H, w.G, (const double *)nullptr);
        hipLaunchKernelGGL(k_pt_l2, dim3(nblocks(4L * g.Vh, kBlock)), block, 0, ctx->stream, g, ctx->Uf, r, sc, w.W,
                           w.G, 1.0, (double2 *)nullptr, w.z, (const double *)nullptr, (const double2 *)nullptr,
                           (double *)nullptr);
        LAUNCHCHK(ctx);
        if (op >= 0) {
            // y = Khat z, d = y - rhat, Gz = Khat d (Khat Hermitian)
            if ((rc = op_apply_K_f32(ctx, op, w.z, ky, kte, kto, nullptr))) return rc;
            hipLaunchKernelGGL(k_pt_resid, grid, block, 0, ctx->stream, g, ky, r, sc, kte, ctx->red);
            LAUNCHCHK(ctx);
            if ((rc = op_apply_K_f32(ctx, op, kte, w.Gz, ky, kto, nullptr))) return rc;
        } else {
            const double2 *e = (const double2 *)E[p];
            double ne = host_norm(ctx, e, &rc);
            if (rc) return rc;
            double neh = (ne / nr) * (ne / nr);
            hipLaunchKernelGGL(k_pt_gz, grid, block, 0, ctx->stream, g, w.z, e, sc, (float)(1.0 / neh), w.Gz,
                               ctx->red);
            LAUNCHCHK(ctx);
        }
        double lp;
        if ((rc = red_finish(ctx, ctx->red, grid.x, 1, &lp))) return rc;
        tot += lp;
        // A2 and A0
        hipLaunchKernelGGL(k_pt_grad2, grid, block, 0, ctx->stream, g, ctx->Uf, r, sc, w.G, w.Gz, w.part);
        col_sums(ctx, w, nwaves, 2 * (NW2 + NW0));
        LAUNCHCHK(ctx);
        HIPCHK(ctx, hipMemcpyAsync(tmp.data(), w.sum, sizeof(double) * 2 * (NW2 + NW0), hipMemcpyDeviceToHost,
                                   ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        for (int k = 0; k < 2 * (NW2 + NW0); k++) acc[2 * NW1 + k] += tmp[k];
        // back through layer 2 and the gate, then A1
        hipLaunchKernelGGL(k_pt_back, grid, block, 0, ctx->stream, g, ctx->Uf, w.W, w.Gz, w.H, w.Gh);
        hipLaunchKernelGGL(k_pt_grad1, grid, block, 0, ctx->stream, g, ctx->Uf, r, sc, w.Gh, w.part);
        col_sums(ctx, w, nwaves, 2 * NW1);
        LAUNCHCHK(ctx);
        HIPCHK(ctx, hipMemcpyAsync(tmp.data(), w.sum, sizeof(double) * 2 * NW1, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        for (int k = 0; k < 2 * NW1; k++) acc[k] += tmp[k];
    }
    *loss = tot;
    for (int k = 0; k < 2 * NW; k++) A[k] = acc[k];
    return 0;
}

// Adam on the real and imaginary parts of the weights, gradient 2 conj(A) from
// pfmp_ptnet_grad over all pairs each step; W updated in place, losses[step] filled.
extern "C" int pfmp_ptnet_train(pfmp_ctx *ctx, double *W, int op, int npairs, const void *const *R,
                                const void *const *E, int steps, double lr, double *losses)
{
    if (!ctx || !W || steps <= 0 || !(lr > 0)) return ctx ? set_err(ctx, PFMP_ERR_ARG, "ptnet_train") : PFMP_ERR_ARG;
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    std::vector<double> m(2 * NW, 0.0), v(2 * NW, 0.0), A(2 * NW);
    for (int s = 0; s < steps; s++) {
        double loss;
        int rc = pfmp_ptnet_grad(ctx, W, op, npairs, R, E, &loss, A.data());
        if (rc) return rc;
        if (losses) losses[s] = loss;
        const double c1 = 1 - std::pow(b1, s + 1), c2 = 1 - std::pow(b2, s + 1);
        for (int k = 0; k < NW; k++) {
            // dL/dRe w = 2 Re A, dL/dIm w = -2 Im A
            double gr[2] = {2 * A[2 * k], -2 * A[2 * k + 1]};
            for (int q = 0; q < 2; q++) {
                int j = 2 * k + q;
                m[j] = b1 * m[j] + (1 - b1) * gr[q];
                v[j] = b2 * v[j] + (1 - b2) * gr[q] * gr[q];
                W[j] -= lr * (m[j] / c1) / (std::sqrt(v[j] / c2) + eps);
            }
        }
    }
    return 0;
}

// Flexible CG on Khat with the network as preconditioner (W = NULL: identity, i.e.
// CG written in the flexible form).  beta = <z+, r+ - r> / <z, r> (Polak-Ribiere).
extern "C" int pfmp_fcg_solve(pfmp_ctx *ctx, int op, const double *W, const void *b_, void *x_,
                              const pfmp_solver_params *prm, pfmp_solver_stats *st)
{
    if (!ctx || !b_ || !x_ || !prm || !(prm->tol > 0) || prm->maxiter <= 0)
        return ctx ? set_err(ctx, PFMP_ERR_ARG, "fcg_solve: bad arguments") : PFMP_ERR_ARG;
    if (op < 0 || op >= PFMP_MAX_OPS || !ctx->ops[op].valid || !ctx->have_gauge)
        return set_err(ctx, PFMP_ERR_STATE, "fcg_solve: operator not configured");
    if (int rc0 = op_ready(ctx, op)) return rc0;
    if (int rc0 = gauge_f32_ready(ctx)) return rc0;
    auto t0 = std::chrono::steady_clock::now();
    const Geom &g = ctx->g;
    const long n = 12L * g.Vh;
    const size_t vb = sizeof(double) * spinor_reals(g);
    PtWs w{};
    int rc;
    if (W && (rc = pt_ws(ctx, W, w))) return rc;
    double2 *r = pool_get(ctx, 2010), *T = pool_get(ctx, 2011), *z = pool_get(ctx, 2012), *p = pool_get(ctx, 2013),
            *q = pool_get(ctx, 2014), *t = pool_get(ctx, 2015);
    if (!r || !T || !z || !p || !q || !t) return set_err(ctx, PFMP_ERR_OOM, "fcg workspace");
    const int nb = op_nparts(g), ndot = 256, nl2 = nblocks(4L * g.Vh, kBlock);
    // part_b holds the |r|^2 block partials (nb) and the two dot products (2 ndot, or
    // 2 per block of the network's second layer)
    long npb = nb;
    if (2L * ndot > npb) npb = 2L * ndot;
    if (2L * nl2 > npb) npb = 2L * nl2;
    double *part_a = (double *)ws_alloc(ctx, sizeof(double) * (nb + 64), 9);
    double *part_b = (double *)ws_alloc(ctx, sizeof(double) * (npb + 64), 10);
    if (!part_a || !part_b) return set_err(ctx, PFMP_ERR_OOM, "fcg workspace");
    const double2 *b = (const double2 *)b_;
    double2 *x = (double2 *)x_;
    double *fs = ctx->scal + kFcgBase;
    OpSlot &s = ctx->ops[op];
    const bool cl = s.csw != 0;
    const double mk2 = -s.kappa * s.kappa;
    dim3 pgrid(nblocks(4L * g.Vh, kBlock)), pblock(kBlock);
    HIPCHK(ctx, hipMemsetAsync(x, 0, vb, ctx->stream));
    {
        const double bn0 = host_norm(ctx, b, &rc);
        if (rc) return rc;
        if (bn0 == 0) {   // b = 0: x = 0 solves it exactly
            if (st) *st = pfmp_solver_stats{};
            return 0;
        }
    }
    HIPCHK(ctx, hipMemcpyAsync(r, b, vb, hipMemcpyDeviceToDevice, ctx->stream));
    if ((rc = launch_norm2(ctx, b, n, ctx->red))) return rc;
    hipLaunchKernelGGL(k_f_init, dim3(1), dim3(kRedBlock), 0, ctx->stream, ctx->red, ctx->nblk_red,
                       prm->tol * prm->tol, prm->maxiter, fs);
    LAUNCHCHK(ctx);
    // z = N(r) (or r), rz = <z, r>, p = z (or the fallback p = r)
    double *dots = nullptr;   // the second layer's <z, r>, <z, q> partials (in the iterations)
    bool use_net = W != nullptr;
    auto precondition = [&]() -> int {
        if (use_net) {
            hipLaunchKernelGGL(k_pt_l1, pgrid, pblock, 0, ctx->stream, g, ctx->Uf, r, 0.f, w.W, (float2 *)nullptr,
                               w.G, (const double *)fs);
            hipLaunchKernelGGL(k_pt_l2, pgrid, pblock, 0, ctx->stream, g, ctx->Uf, r, 0.f, w.W, w.G, 0.0, z,
                               (float2 *)nullptr, (const double *)fs, (const double2 *)q, dots);
            LAUNCHCHK(ctx);
            if (dots) return launch_total<2>(ctx, dots, nl2, fs + F_ZR, fs + F_DONE);
            return 0;
        }
        HIPCHK(ctx, hipMemcpyAsync(z, r, vb, hipMemcpyDeviceToDevice, ctx->stream));
        return 0;
    };
    if ((rc = precondition())) return rc;
    hipLaunchKernelGGL(k_f_dots, dim3(ndot), dim3(kBlock), 0, ctx->stream, n, z, r, z, fs, part_b);
    hipLaunchKernelGGL(k_f_beta, dim3(1), dim3(kRedBlock), 0, ctx->stream, part_b, ndot, 1, fs);
    hipLaunchKernelGGL(k_f_update_p, dim3(nblocks(n, 256)), dim3(256), 0, ctx->stream, n, z, r, p, fs);
    LAUNCHCHK(ctx);
    const int chunk = prm->check_every > 0 ? prm->check_every : 10;
    double h[F_NSLOT];
    // one iteration: fixed launches, replayed as a graph
    auto iteration = [&]() -> int {
        int e;
        // <p, Khat p> = |Mhat p|^2 partials, then q = Khat p fused with the x, r updates
        if ((e = clovinv64(ctx, 1, p, s.clov[1], T, 1.0, 1.0, cl, fs + F_DONE))) return e;
        if ((e = xpay64(ctx, 0, p, T, s.clov[0], mk2, t, 1.0, cl, part_a, fs + F_DONE))) return e;
        if ((e = launch_total<1>(ctx, part_a, nb, fs + F_PQ, fs + F_DONE))) return e;
        if ((e = clovinv64(ctx, 1, t, s.clov[1], T, -1.0, 1.0, cl, fs + F_DONE))) return e;
#define FHOP4(CL, LM)                                                                                        \
    hipLaunchKernelGGL((k_f_hop4<CL, LM>), dim3(nb), dim3(kBlock), 0, ctx->stream, g, t, T, ctx->U, s.clov[0], mk2, \
                       p, q, x, r, fs, part_b)
#define FHOP4_1(LM) FHOP4(1, LM)
#define FHOP4_0(LM) FHOP4(0, LM)
        if (cl) { PFMP_LM_SWITCH(link_mode(g), FHOP4_1) }
        else { PFMP_LM_SWITCH(link_mode(g), FHOP4_0) }
#undef FHOP4_1
#undef FHOP4_0
#undef FHOP4
        hipLaunchKernelGGL(k_f_norm, dim3(1), dim3(kFinishThreads), 0, ctx->stream, part_b, nb, fs);
        LAUNCHCHK(ctx);
        if (use_net) {
            // z = N(r) with <z, r> and <z, q>, then beta and p in one launch
            dots = part_b;
            e = precondition();
            dots = nullptr;
            if (e) return e;
            hipLaunchKernelGGL(k_f_update_p_fused, dim3(nblocks(n, kRedBlock)), dim3(kRedBlock), 0, ctx->stream, n, z,
                               r, p, fs);
        } else {
            // identity: z = r is read directly
            hipLaunchKernelGGL(k_f_dots, dim3(ndot), dim3(kBlock), 0, ctx->stream, n, r, r, q, fs, part_b);
            hipLaunchKernelGGL(k_f_beta, dim3(1), dim3(kRedBlock), 0, ctx->stream, part_b, ndot, 0, fs);
            hipLaunchKernelGGL(k_f_update_p, dim3(nblocks(n, 256)), dim3(256), 0, ctx->stream, n, r, r, p, fs);
        }
        LAUNCHCHK(ctx);
        return 0;
    };
    auto make_key = [&](bool net) {
        std::vector<uint64_t> key;
        key_add(key, 4);   // flexible-CG iteration
        key_geom(key, g);
        for (const void *ptr : {(const void *)p, (const void *)T, (const void *)t, (const void *)q, (const void *)x,
                                (const void *)r, (const void *)z, (const void *)part_a, (const void *)part_b,
                                (const void *)fs, (const void *)ctx->U, (const void *)ctx->Uf,
                                (const void *)s.clov[0], (const void *)s.clov[1],
                                (const void *)(net ? w.W : nullptr), (const void *)(net ? w.G : nullptr)})
            key_add(key, ptr);
        key_add(key, mk2);
        key_add(key, (int)cl);
        return key;
    };
    // Plain CG stays the fallback of the whole solve: when the network has not cut
    // |r| by 2 within kFcgStall iterations, the solve goes on as plain CG from the
    // current iterate (p = r), so a poor network costs at most kFcgStall iterations
    // more than the plain method from there.
    constexpr int kFcgStall = 100;
    double rr_ref = -1, it_ref = 0, it_switch = -1;
    for (;;) {
        if ((rc = graph_run(ctx, make_key(use_net), chunk, iteration))) return rc;
        HIPCHK(ctx, hipMemcpyAsync(ctx->red_host, fs, sizeof(double) * F_NSLOT, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        for (int k = 0; k < F_NSLOT; k++) h[k] = ctx->red_host[k];
        if (h[F_DONE] != 0) break;
        if (!use_net) continue;
        if (rr_ref < 0 || h[F_RN2] < 0.25 * rr_ref) {
            rr_ref = h[F_RN2];
            it_ref = h[F_ITER];
        } else if (h[F_ITER] - it_ref >= kFcgStall) {
            use_net = false;
            it_switch = h[F_ITER];
            hipLaunchKernelGGL(k_f_dots, dim3(ndot), dim3(kBlock), 0, ctx->stream, n, r, r, r, fs, part_b);
            hipLaunchKernelGGL(k_f_beta, dim3(1), dim3(kRedBlock), 0, ctx->stream, part_b, ndot, 1, fs);
            hipLaunchKernelGGL(k_f_update_p, dim3(nblocks(n, 256)), dim3(256), 0, ctx->stream, n, r, r, p, fs);
            LAUNCHCHK(ctx);
        }
    }
    // FP64 true residual
    if ((rc = op_apply_K(ctx, op, x, q, t, T, nullptr))) return rc;
    HIPCHK(ctx, hipMemcpyAsync(r, b, vb, hipMemcpyDeviceToDevice, ctx->stream));
    double m1[2] = {-1.0, 0.0}, p1[2] = {1.0, 0.0};
    if ((rc = pfmp_axpby(ctx, m1, q, p1, r))) return rc;
    double bn = host_norm(ctx, b, &rc);
    if (rc) return rc;
    double tr = host_norm(ctx, r, &rc);
    if (rc) return rc;
    auto t1 = std::chrono::steady_clock::now();
    if (st) {
        st->iters = (int)h[F_ITER];
        // plain-CG steps: the per-step fallbacks and every step after a switch to plain CG
        st->reliable_updates = (int)h[F_NFB] + (it_switch >= 0 ? (int)(h[F_ITER] - it_switch) : 0);
        st->true_res = bn > 0 ? tr / bn : 0;
        st->seconds = std::chrono::duration<double>(t1 - t0).count();
        st->kmults = (int)h[F_ITER] + 1;
    }
    if (!(tr <= prm->tol * bn)) return set_err(ctx, PFMP_ERR_NOCONV, "fcg_solve: maxiter reached");
    return 0;
}

// CG on Khat recording (x_k, r_k) at the requested iterations (ascending), so that
// training pairs (r_k, e_k = x - x_k) can be formed once the solve has converged.
// Host-driven textbook CG in FP64; returns the number of snapshots taken.
extern "C" int pfmp_cg_harvest(pfmp_ctx *ctx, int op, const void *b_, void *x_, double tol, int maxiter, int nsnap,
                               const int *snap_iters, void *const *snap_x, void *const *snap_r, int *ntaken)
{
    if (!ctx || !b_ || !x_ || (nsnap > 0 && (!snap_iters || !snap_x || !snap_r)) || !ntaken)
        return ctx ? set_err(ctx, PFMP_ERR_ARG, "cg_harvest: bad arguments") : PFMP_ERR_ARG;
    if (op < 0 || op >= PFMP_MAX_OPS || !ctx->ops[op].valid || !ctx->have_gauge)
        return set_err(ctx, PFMP_ERR_STATE, "cg_harvest: operator not configured");
    if (int rc0 = op_ready(ctx, op)) return rc0;
    const Geom &g = ctx->g;
    const long n = 12L * g.Vh;
    const size_t vb = sizeof(double) * spinor_reals(g);
    double2 *r = pool_get(ctx, 2010), *p = pool_get(ctx, 2013), *q = pool_get(ctx, 2014), *te = pool_get(ctx, 2015),
            *to = pool_get(ctx, 2016);
    if (!r || !p || !q || !te || !to) return set_err(ctx, PFMP_ERR_OOM, "harvest workspace");
    const int nb = op_nparts(g);
    double *part = (double *)ws_alloc(ctx, sizeof(double) * (nb + 64), 9);
    if (!part) return set_err(ctx, PFMP_ERR_OOM, "harvest workspace");
    const double2 *b = (const double2 *)b_;
    double2 *x = (double2 *)x_;
    int rc;
    HIPCHK(ctx, hipMemsetAsync(x, 0, vb, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(r, b, vb, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(p, b, vb, hipMemcpyDeviceToDevice, ctx->stream));
    double bn = host_norm(ctx, b, &rc);
    if (rc) return rc;
    double rr = bn * bn;
    int k = 0, s = 0;
    while (rr > tol * tol * bn * bn && k < maxiter) {
        if (s < nsnap && snap_iters[s] == k) {
            HIPCHK(ctx, hipMemcpyAsync(snap_x[s], x, vb, hipMemcpyDeviceToDevice, ctx->stream));
            HIPCHK(ctx, hipMemcpyAsync(snap_r[s], r, vb, hipMemcpyDeviceToDevice, ctx->stream));
            s++;
        }
        if ((rc = op_apply_K(ctx, op, p, q, te, to, part))) return rc;
        double pq;
        if ((rc = red_finish(ctx, part, nb, 1, &pq))) return rc;
        double alpha = rr / pq;
        double al[2] = {alpha, 0}, one[2] = {1, 0}, mal[2] = {-alpha, 0};
        if ((rc = pfmp_axpby(ctx, al, p, one, x))) return rc;
        if ((rc = pfmp_axpby(ctx, mal, q, one, r))) return rc;
        double rn = host_norm(ctx, r, &rc);
        if (rc) return rc;
        double beta = rn * rn / rr;
        rr = rn * rn;
        double be[2] = {beta, 0};
        if ((rc = pfmp_axpby(ctx, one, r, be, p))) return rc;
        k++;
    }
    (void)n;
    *ntaken = s;
    return k >= maxiter ? set_err(ctx, PFMP_ERR_NOCONV, "cg_harvest: maxiter reached") : 0;
}
