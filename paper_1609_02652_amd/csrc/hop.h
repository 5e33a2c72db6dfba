// hop.h -- device building blocks of the Wilson hopping term and the clover
// apply, shared by the operator kernels and the fused solver kernels.
//
// Two lanes per output site (see "two lanes per site" below).  For each of the 8
// directions the neighbour spinor is spin-projected to a half spinor, multiplied by
// the link and added back; projectors in the chiral basis, g_mu = [[0, B],[C, 0]]
// with B = C^-1:
//   (1 + s g_mu) psi = [h ; s C h],  h = psi_up + s B psi_low,   s = -1 (forward), +1 (backward)
// with B = -i sigma_k, C = i sigma_k for k = x,y,z and B = C = 1 for t.
// Neighbour indices come from the site coordinates (no index tables are read).
#pragma once
#include <hip/hip_fp16.h>

#include "internal.h"

// FP16 records: three half2 (12 bytes) that one lane moves with a single dwordx3 load or
// store.  Every FP16 field is laid out in such records, so a lane issues a quarter as many
// memory instructions as with one half2 plane per component, and each instruction carries
// three times the bytes: the loads in flight per wave, not the bytes, bound the FP16
// stencils on a lattice larger than the last-level cache.
struct __attribute__((aligned(4))) H3 {
    __half2 v[3];
};

// FP16 spinor storage (one parity): the 3 colours of spin g of site i in record
// h[g * Vh + i] (4 x 12 B per site), then one FP32 scale per site; the stored values are
// v / scale with scale = max |Re|, |Im| over the site's 24 reals (IEEE binary16, round to
// nearest even), arithmetic in FP32.
struct HalfField {
    H3 *h;
    float *s;
};

__device__ __forceinline__ void load_spinor(const HalfField &f, int Vh, int i, float gs, float2 *v)
{
    const float sc = f.s[i];
#pragma unroll
    for (int sp = 0; sp < 4; sp++) {
        const H3 q = f.h[(long)sp * Vh + i];
        const float m = sp < 2 ? sc : sc * gs;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const float2 x = __half22float2(q.v[a]);
            v[3 * sp + a] = make_float2(x.x * m, x.y * m);
        }
    }
}

__device__ __forceinline__ void store_spinor(const HalfField &f, int Vh, int i, float gs, const float2 *v)
{
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 12; k++) m = fmaxf(m, fmaxf(fabsf(v[k].x), fabsf(v[k].y)));
    const float inv = m > 0.f ? 1.f / m : 0.f;
    f.s[i] = m;
#pragma unroll
    for (int sp = 0; sp < 4; sp++) {
        const float q = sp < 2 ? inv : inv * gs;
        H3 r;
#pragma unroll
        for (int a = 0; a < 3; a++) r.v[a] = __floats2half2_rn(v[3 * sp + a].x * q, v[3 * sp + a].y * q);
        f.h[(long)sp * Vh + i] = r;
    }
}

// load a spinor (12 complex) of site i; gs = -1 flips the lower spins (g5)
template <typename C>
__device__ __forceinline__ void load_spinor(const C *__restrict__ f, int Vh, int i, decltype(C::x) gs, C *v)
{
#pragma unroll
    for (int k = 0; k < 12; k++) {
        C a = f[(long)k * Vh + i];
        v[k] = k < 6 ? a : cscale(a, gs);
    }
}

template <typename C>
__device__ __forceinline__ void store_spinor(C *__restrict__ f, int Vh, int i, decltype(C::x) gs, const C *v)
{
#pragma unroll
    for (int k = 0; k < 12; k++) f[(long)k * Vh + i] = k < 6 ? v[k] : cscale(v[k], gs);
}

// h = psi_up + s B psi_low (per colour), for direction MU and sign S
template <int MU, int S, typename C>
__device__ __forceinline__ void project(const C *p, C *h)
{
#pragma unroll
    for (int a = 0; a < 3; a++) {
        C p0 = p[a], p1 = p[3 + a], p2 = p[6 + a], p3 = p[9 + a];
        if (MU == 0) {          // B p_low = (-i p3, -i p2)
            h[a] = S < 0 ? cadd(p0, ctimesi(p3)) : csub(p0, ctimesi(p3));
            h[3 + a] = S < 0 ? cadd(p1, ctimesi(p2)) : csub(p1, ctimesi(p2));
        } else if (MU == 1) {   // B p_low = (-p3, p2)
            h[a] = S < 0 ? cadd(p0, p3) : csub(p0, p3);
            h[3 + a] = S < 0 ? csub(p1, p2) : cadd(p1, p2);
        } else if (MU == 2) {   // B p_low = (-i p2, i p3)
            h[a] = S < 0 ? cadd(p0, ctimesi(p2)) : csub(p0, ctimesi(p2));
            h[3 + a] = S < 0 ? csub(p1, ctimesi(p3)) : cadd(p1, ctimesi(p3));
        } else {                // B p_low = (p2, p3)
            h[a] = S < 0 ? csub(p0, p2) : cadd(p0, p2);
            h[3 + a] = S < 0 ? csub(p1, p3) : cadd(p1, p3);
        }
    }
}

// ------------------------------------------------------------------ two lanes per site
//
// The operator kernels run two lanes per output site (a lane pair in one wavefront).
// Lane hb of the pair owns chiral block hb (spins 2hb, 2hb+1) of the result.  For the
// hop it projects only half-spin hb of every neighbour: with partner lower spin q,
//   h = psi_hb + S f psi_q,  f = sgp (i or 1),   q = 3 - hb (mu = x, y), 2 + hb (mu = z, t),
// multiplies one SU(3) vector, adds it to its upper spin hb and S r w to lower spin q:
//   mu = x: f = -i,            r = i
//   mu = y: f = r = (hb ? 1 : -1)
//   mu = z: f = (hb ? i : -i), r = -f
//   mu = t: f = r = 1
// (the chiral-basis projectors written per half-spin).  The two partial lower spins
// are combined by one lane swap at the end (hop_pair).

template <int IM, typename C>
__device__ __forceinline__ C unit_mul(C v, decltype(C::x) sg)
{
    return IM ? mk<C>(-sg * v.y, sg * v.x) : mk<C>(sg * v.x, sg * v.y);
}

// Streaming (non-temporal) load: every link is read once per hop launch, so it should
// not displace the neighbour spinors, which are read eight times, from the caches.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream(const double2 *p)
{
    nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2 *>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_stream(const float2 *p)
{
    nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2 *>(p));
    return make_float2(v.x, v.y);
}

// Link storage: a pointer to complex planes of the arithmetic type (FP64), the FP32 copy or the
// FP16 copy (HalfLinks; SU(3) entries have |u| <= 1, so binary16 needs no scale) read into
// FP32.  lload / lstream fetch element idx of the planes (lstream non-temporally); lshift
// offsets the base.  Both copies keep the offsets of the complex planes of one link (9 Vh
// complex per link), but within a link row r of site i is the record of 3 complex at complex
// 3 r Vh + 3 i (24 bytes in FP32, 12 in FP16).
struct HalfLinks {
    const __half2 *p;
};
template <typename C> __device__ __forceinline__ C lload(const C *__restrict__ U, long idx) { return U[idx]; }
template <typename C> __device__ __forceinline__ C lstream(const C *__restrict__ U, long idx) { return ld_stream(U + idx); }
template <typename C> __device__ __forceinline__ const C *lshift(const C *U, long off) { return U + off; }
__device__ __forceinline__ HalfLinks lshift(const HalfLinks &U, long off) { return HalfLinks{U.p + off}; }

// ------------------------------------------------------------------ leg pipeline
//
// One leg is one of the 8 hops (direction mu, forward or backward): the neighbour's
// half-spin hb and partner lower spin q, and the link.  Its operands are first loaded
// raw (FP16 stays packed) into a Leg, and only later decoded and applied, so that the
// loads of PD legs are in flight while one is computed.  With a single leg in flight
// every hop waits for 8 memory round trips in a row, which bounds the kernel whenever the
// lattice gives each SIMD only a few waves (16^3 x 32: two per SIMD).  The arithmetic and
// its order are the same for every PD.

template <typename C, typename In>
struct SpinLeg {
    C v[6];
    __device__ __forceinline__ void load(const In f, long Vh, int j, int k0, int k1)
    {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            v[a] = f[(long)(k0 + a) * Vh + j];
            v[3 + a] = f[(long)(k1 + a) * Vh + j];
        }
    }
    __device__ __forceinline__ C raw(int k) const { return v[k]; }
    __device__ __forceinline__ decltype(C::x) scale() const { return 1; }
};
// FP16: raw() gives the stored values, scale() the site's factor; the two spins are one
// record each (k0 and k1 are multiples of 3)
template <>
struct SpinLeg<float2, HalfField> {
    H3 v[2];
    float s;
    __device__ __forceinline__ void load(const HalfField &f, long Vh, int j, int k0, int k1)
    {
        v[0] = f.h[(long)(k0 / 3) * Vh + j];
        v[1] = f.h[(long)(k1 / 3) * Vh + j];
        s = f.s[j];
    }
    __device__ __forceinline__ float2 raw(int k) const { return __half22float2(v[k / 3].v[k % 3]); }
    __device__ __forceinline__ float scale() const { return s; }
};

// N link planes (6 with the third row rebuilt, else 9); ST: streaming loads
template <typename C, typename UL, int N>
struct LinkLeg {
    C u[N];
    template <int ST>
    __device__ __forceinline__ void load(UL U, long stride, long site)
    {
#pragma unroll
        for (int k = 0; k < N; k++) u[k] = ST ? lstream<C>(U, k * stride + site) : lload<C>(U, k * stride + site);
    }
    __device__ __forceinline__ C get(int k) const { return u[k]; }
};
// FP32 links: one 24-byte record per row (a dwordx4 and a dwordx2 load).  The loads stay
// cached in every link mode: at 32^3 x 64 non-temporal record loads made the FP32 CG
// iteration 4 % and the FP16-storage one with FP32 links 5 % slower than cached ones.
struct __attribute__((aligned(8))) F3 {
    float2 v[3];
};
template <int N>
struct LinkLeg<float2, const float2 *, N> {
    F3 u[N / 3];
    template <int ST>
    __device__ __forceinline__ void load(const float2 *U, long stride, long site)
    {
#pragma unroll
        for (int r = 0; r < N / 3; r++) u[r] = reinterpret_cast<const F3 *>(U + 3 * r * stride)[site];
    }
    __device__ __forceinline__ float2 get(int k) const { return u[k / 3].v[k % 3]; }
};
// FP16 links: one record per row (N / 3 rows)
template <int N>
struct LinkLeg<float2, HalfLinks, N> {
    H3 u[N / 3];
    template <int ST>
    __device__ __forceinline__ void load(const HalfLinks &U, long stride, long site)
    {
#pragma unroll
        for (int r = 0; r < N / 3; r++) u[r] = reinterpret_cast<const H3 *>(U.p + 3 * r * stride)[site];
    }
    __device__ __forceinline__ float2 get(int k) const { return __half22float2(u[k / 3].v[k % 3]); }
};

// LM (link mode): bit 0 rebuild the third row, bit 1 streaming loads
template <typename C, typename In, typename UL, int LM>
struct Leg {
    SpinLeg<C, In> sp;
    LinkLeg<C, UL, (LM & 1) ? 6 : 9> lk;
    decltype(C::x) sg;   // boundary sign of the hop
};

// legs in flight per lane: all 8 for FP16 storage (13 registers per leg); for FP32 and
// FP64 fewer, as their legs take 2x and 4x the registers
#ifndef PFMP_LEGS_F16
#define PFMP_LEGS_F16 8
#endif
#ifndef PFMP_LEGS_F32
#define PFMP_LEGS_F32 4
#endif
#ifndef PFMP_LEGS_F64
#define PFMP_LEGS_F64 2
#endif
template <typename In> struct LegDepth { static constexpr int value = PFMP_LEGS_F64; };
template <> struct LegDepth<HalfField> { static constexpr int value = PFMP_LEGS_F16; };
template <> struct LegDepth<const float2 *> { static constexpr int value = PFMP_LEGS_F32; };
template <> struct LegDepth<float2 *> { static constexpr int value = PFMP_LEGS_F32; };

template <int MU, int DIR, int LM, typename C, typename In, typename UL>
__device__ __forceinline__ void leg_load(const Geom &g, int pout, int i, const int *c, int hb, const In in, UL U,
                                         Leg<C, In, UL, LM> &l)
{
    int s;
    const int j = eo_neighbour(g, c, MU, DIR ? -1 : +1, &s);
    const int q = MU < 2 ? 3 - hb : 2 + hb;
    l.sp.load(in, g.Vh, j, 3 * hb, 3 * q);
    // forward: U_mu(x) on the output parity; backward: U_mu(x - mu) on the other one
    const int lp = DIR ? 1 - pout : pout;
    l.lk.template load<(LM >> 1) & 1>(lshift(U, ((long)(lp * 4 + MU) * 9) * g.Vh), g.Vh, DIR ? j : i);
    l.sg = (decltype(C::x))s;
}

// w = U h (DIR = 0) or U^dag h (DIR = 1) for one half-spin (3 colours).  With recon the
// link is in SU(3) and its third row is the conjugate cross product of the first two.
template <int DIR, int LM, typename C, typename LL>
__device__ __forceinline__ void leg_su3(const LL &L, const C *h, C *w)
{
    C u[9];
#pragma unroll
    for (int k = 0; k < 6; k++) u[k] = L.get(k);
    if constexpr ((LM & 1) != 0) {
        u[6] = cconj(csub(cmul(u[1], u[5]), cmul(u[2], u[4])));
        u[7] = cconj(csub(cmul(u[2], u[3]), cmul(u[0], u[5])));
        u[8] = cconj(csub(cmul(u[0], u[4]), cmul(u[1], u[3])));
    } else {
#pragma unroll
        for (int k = 6; k < 9; k++) u[k] = L.get(k);
    }
#pragma unroll
    for (int a = 0; a < 3; a++) {
        C acc = mk<C>(0, 0);
#pragma unroll
        for (int b = 0; b < 3; b++) {
            if (DIR) cfmac(acc, u[3 * b + a], h[b]);
            else cfma(acc, u[3 * a + b], h[b]);
        }
        w[a] = acc;
    }
}

// forward leg: (1 - g_mu) U_mu(x) psi(x + mu); backward: (1 + g_mu) U_mu(x - mu)^dag psi(x - mu)
template <int MU, int DIR, int LM, typename C, typename LegT>
__device__ __forceinline__ void leg_apply(const LegT &l, int hb, decltype(C::x) gs, C *up, C *loA, C *loB)
{
    using R = decltype(C::x);
    constexpr int IM = (MU == 0 || MU == 2) ? 1 : 0;
    const R sgp = MU == 0 ? (R)-1 : (MU == 3 ? (R)1 : (hb ? (R)1 : (R)-1));
    const R sgr = MU == 0 ? (R)1 : (MU == 2 ? -sgp : sgp);
    C *lo = MU < 2 ? loA : loB;
    // The signs (all +-1) are combined before they meet the data, so each costs nothing per
    // component; the neighbour's FP16 scale and the boundary sign multiply U h once.
    const R fq = sgp * gs;
    const R fu = l.sg * l.sp.scale(), fl = fu * sgr;
    C h[3], w[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const C pt = l.sp.raw(a), pq = l.sp.raw(3 + a);
        h[a] = DIR ? cadd(pt, unit_mul<IM>(pq, fq)) : csub(pt, unit_mul<IM>(pq, fq));
    }
    leg_su3<DIR, LM>(l.lk, h, w);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        up[a] = cadd(up[a], cscale(w[a], fu));
        lo[a] = DIR ? cadd(lo[a], unit_mul<IM>(w[a], fl)) : csub(lo[a], unit_mul<IM>(w[a], fl));
    }
}

// apply leg L from slot L % PD, then refill that slot with leg L + PD
template <int L, int PD, int LM, typename C, typename In, typename UL>
__device__ __forceinline__ void hop_legs(const Geom &g, int pout, int i, const int *c, int hb, const In in, UL U,
                                         decltype(C::x) gs, Leg<C, In, UL, LM> *buf, C *up, C *loA, C *loB)
{
    if constexpr (L < 8) {
        leg_apply<(L >> 1), (L & 1), LM, C>(buf[L % PD], hb, gs, up, loA, loB);
        if constexpr (L + PD < 8) {
            leg_load<((L + PD) >> 1), ((L + PD) & 1), LM, C>(g, pout, i, c, hb, in, U, buf[L % PD]);
            // keep the scheduler from sinking the loads to their first use
            __builtin_amdgcn_sched_barrier(0);
        }
        hop_legs<L + 1, PD, LM, C>(g, pout, i, c, hb, in, U, gs, buf, up, loA, loB);
    }
}

template <int L, int PD, int LM, typename C, typename In, typename UL>
__device__ __forceinline__ void hop_prime(const Geom &g, int pout, int i, const int *c, int hb, const In in, UL U,
                                          Leg<C, In, UL, LM> *buf)
{
    if constexpr (L < PD) {
        leg_load<(L >> 1), (L & 1), LM, C>(g, pout, i, c, hb, in, U, buf[L]);
        hop_prime<L + 1, PD, LM, C>(g, pout, i, c, hb, in, U, buf);
    }
}

__device__ __forceinline__ double pair_swap(double v) { return __shfl_xor(v, 1, 64); }
__device__ __forceinline__ float pair_swap(float v) { return __shfl_xor(v, 1, 64); }

// D_hop in (gs = -1 flips the lower spins of the input), chiral block hb of the
// result at output site i of parity pout; LM: link mode (see Leg)
template <int LM, typename C, typename In, typename UL, int PD = LegDepth<In>::value>
__device__ __forceinline__ void hop_pair(const Geom &g, int pout, int i, int hb, const In in, UL U,
                                         decltype(C::x) gs, C *blk)
{
    int c[4];
    eo_coords(g, pout, i, c);
    C up[3], loA[3], loB[3];   // upper spin hb; lower spins 3 - hb and 2 + hb
#pragma unroll
    for (int a = 0; a < 3; a++) up[a] = loA[a] = loB[a] = mk<C>(0, 0);
    Leg<C, In, UL, LM> buf[PD];
    hop_prime<0, PD, LM, C>(g, pout, i, c, hb, in, U, buf);
    __builtin_amdgcn_sched_barrier(0);
    hop_legs<0, PD, LM, C>(g, pout, i, c, hb, in, U, gs, buf, up, loA, loB);
    // lane 0 keeps spin 0 and takes spin 1 from lane 1; lane 1 sums the lower spins
    C x[6];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        x[a] = hb ? up[a] : loB[a];       // lane 0 sends its share of spin 2
        x[3 + a] = hb ? up[a] : loA[a];   // ... and of spin 3
    }
#pragma unroll
    for (int k = 0; k < 6; k++) x[k] = mk<C>(pair_swap(x[k].x), pair_swap(x[k].y));
#pragma unroll
    for (int a = 0; a < 3; a++) {
        blk[a] = hb ? cadd(loA[a], x[a]) : up[a];
        blk[3 + a] = hb ? cadd(loB[a], x[3 + a]) : x[a];
    }
}

// components 6 hb .. 6 hb + 5 of a spinor; gs scales them when hb = 1 (lower spins)
template <typename C>
__device__ __forceinline__ void load_block(const C *__restrict__ f, int Vh, int i, int hb, decltype(C::x) gs, C *v)
{
#pragma unroll
    for (int k = 0; k < 6; k++) {
        C a = f[(long)(6 * hb + k) * Vh + i];
        v[k] = hb ? cscale(a, gs) : a;
    }
}
__device__ __forceinline__ void load_block(const HalfField &f, int Vh, int i, int hb, float gs, float2 *v)
{
    const float sc = hb ? f.s[i] * gs : f.s[i];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const H3 q = f.h[(long)(2 * hb + h) * Vh + i];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const float2 x = __half22float2(q.v[a]);
            v[3 * h + a] = make_float2(x.x * sc, x.y * sc);
        }
    }
}

template <typename C>
__device__ __forceinline__ void store_block(C *__restrict__ f, int Vh, int i, int hb, decltype(C::x) gs, const C *v)
{
#pragma unroll
    for (int k = 0; k < 6; k++) f[(long)(6 * hb + k) * Vh + i] = hb ? cscale(v[k], gs) : v[k];
}
// FP16 storage: the per-site scale is the maximum over both lanes' blocks
__device__ __forceinline__ void store_block(const HalfField &f, int Vh, int i, int hb, float gs, const float2 *v)
{
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 6; k++) m = fmaxf(m, fmaxf(fabsf(v[k].x), fabsf(v[k].y)));
    m = fmaxf(m, pair_swap(m));
    const float inv = m > 0.f ? 1.f / m : 0.f;
    if (hb == 0) f.s[i] = m;
    const float q = hb ? inv * gs : inv;
#pragma unroll
    for (int h = 0; h < 2; h++) {
        H3 r;
#pragma unroll
        for (int a = 0; a < 3; a++) r.v[a] = __floats2half2_rn(v[3 * h + a].x * q, v[3 * h + a].y * q);
        f.h[(long)(2 * hb + h) * Vh + i] = r;
    }
}

// out[6] = (6x6 Hermitian block b of the clover field at site i) v[6]
// Clover storage: FP64 real planes (12 diagonal planes [b * 6 + k][Vh], then 30 complex
// upper-triangle planes [b * 15 + m][Vh]); the FP32 copy as one 144-byte record per block
// and site (6 diagonal reals, then the 15 complex entries); or the FP16 copy (HalfClover,
// entries of A and A^-1 are O(1)) read into FP32: one 72-byte record of 6 H3 per block and
// site at p[(2 i + b) * 6], the 6 diagonal reals as 3 half2, then the 15 complex entries.
struct HalfClover {
    const H3 *p;
};
template <typename R, typename C>
__device__ __forceinline__ void clover_fetch(const R *__restrict__ cl, int Vh, int i, int b, R *d, C *o)
{
#pragma unroll
    for (int k = 0; k < 6; k++) d[k] = cl[(long)(b * 6 + k) * Vh + i];
    const C *off = reinterpret_cast<const C *>(cl + 12L * Vh);
#pragma unroll
    for (int m = 0; m < 15; m++) o[m] = off[(long)(b * 15 + m) * Vh + i];
}
// FP32 clover: one record of 36 floats per block and site at (2 i + b) * 36, read as nine
// 16-byte loads
__device__ __forceinline__ void clover_fetch(const float *__restrict__ cl, int, int i, int b, float *d, float2 *o)
{
    float f[36];
    const float4 *rf = reinterpret_cast<const float4 *>(cl) + (2L * i + b) * 9;
#pragma unroll
    for (int u = 0; u < 9; u++) {
        const float4 v = rf[u];
        f[4 * u] = v.x; f[4 * u + 1] = v.y; f[4 * u + 2] = v.z; f[4 * u + 3] = v.w;
    }
#pragma unroll
    for (int k = 0; k < 6; k++) d[k] = f[k];
#pragma unroll
    for (int m = 0; m < 15; m++) o[m] = make_float2(f[6 + 2 * m], f[7 + 2 * m]);
}
__device__ __forceinline__ void clover_fetch(const HalfClover &cl, int, int i, int b, float *d, float2 *o)
{
    H3 q[6];
    const H3 *rec = cl.p + (long)(2 * i + b) * 6;
#pragma unroll
    for (int u = 0; u < 6; u++) q[u] = rec[u];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const float2 x = __half22float2(q[0].v[a]);
        d[2 * a] = x.x;
        d[2 * a + 1] = x.y;
    }
#pragma unroll
    for (int m = 0; m < 15; m++) o[m] = __half22float2(q[1 + m / 3].v[m % 3]);
}

// Non-temporal variants (ST = 1) for data a launch touches once: on lattices whose links
// stream (the gauge field beyond the last-level cache) the outputs and the site-local inputs
// of the stencil kernels go the same way, leaving L2 to the neighbour spinors, which are read
// up to eight times (32^3 x 64: FP64 hop 280 -> 259 us, the same bits).  FP16 records keep
// cached accesses.
__device__ __forceinline__ void st_stream(double2 *p, double2 v)
{
    nt_d2 w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<nt_d2 *>(p));
}
__device__ __forceinline__ void st_stream(float2 *p, float2 v)
{
    nt_f2 w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<nt_f2 *>(p));
}
template <int ST, typename C>
__device__ __forceinline__ C ld_st(const C *p)
{
    return ST ? ld_stream(p) : *p;
}
template <int ST, typename C>
__device__ __forceinline__ void st_st(C *p, C v)
{
    if (ST) st_stream(p, v);
    else *p = v;
}
template <int ST, typename C>
__device__ __forceinline__ void load_block_st(const C *__restrict__ f, int Vh, int i, int hb, decltype(C::x) gs, C *v)
{
#pragma unroll
    for (int k = 0; k < 6; k++) {
        C a = ld_st<ST>(f + (long)(6 * hb + k) * Vh + i);
        v[k] = hb ? cscale(a, gs) : a;
    }
}
template <int ST>
__device__ __forceinline__ void load_block_st(const HalfField &f, int Vh, int i, int hb, float gs, float2 *v)
{
    load_block(f, Vh, i, hb, gs, v);
}
template <int ST, typename C>
__device__ __forceinline__ void store_block_st(C *__restrict__ f, int Vh, int i, int hb, decltype(C::x) gs, const C *v)
{
#pragma unroll
    for (int k = 0; k < 6; k++) st_st<ST>(f + (long)(6 * hb + k) * Vh + i, hb ? cscale(v[k], gs) : v[k]);
}
template <int ST>
__device__ __forceinline__ void store_block_st(const HalfField &f, int Vh, int i, int hb, float gs, const float2 *v)
{
    store_block(f, Vh, i, hb, gs, v);
}

// out = (block with diagonal d and upper triangle o) v
template <typename R, typename C>
__device__ __forceinline__ void clover_mul(const R *d, const C *o, const C *v, C *out)
{
#pragma unroll
    for (int r = 0; r < 6; r++) out[r] = cscale(v[r], d[r]);
    int m = 0;
#pragma unroll
    for (int r = 0; r < 6; r++)
#pragma unroll
        for (int q = r + 1; q < 6; q++, m++) {
            cfma(out[r], o[m], v[q]);
            cfmac(out[q], o[m], v[r]);
        }
}

template <typename R, typename C, typename CL>
__device__ __forceinline__ void clover_block(CL cl, int Vh, int i, int b, const C *v, C *out)
{
    R d[6];
    C o[15];
    clover_fetch(cl, Vh, i, b, d, o);
    clover_mul(d, o, v, out);
}

template <typename R, typename C, typename CL>
__device__ __forceinline__ void clover_apply(CL cl, int Vh, int i, const C *v, C *out)
{
    clover_block<R, C>(cl, Vh, i, 0, v, out);
    clover_block<R, C>(cl, Vh, i, 1, v + 6, out + 6);
}

template <typename C, int NW = kBlock / 64>
__device__ __forceinline__ void block_sum_store(double v, double *partials)
{
    __shared__ double sh[NW];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
        for (int k = 0; k < NW; k++) s += sh[k];
        partials[blockIdx.x] = s;
    }
}

// ------------------------------------------------------------------ deterministic totals
//
// A grid-wide sum is written as block partials by the kernel that produces it and
// totalled by one fixed order, the same wherever the total is formed: chunk c of 64
// consecutive partials is reduced by one wave (shuffle tree), and the chunk sums are added
// by 128 lanes (lane k takes chunks k, k + 128, ... in turn, then a shuffle tree per wave
// and the two waves in order).  Trailing zero partials (padding workgroups) leave it
// unchanged.  With few partials every workgroup of the consuming kernel forms the total
// itself (no launch in between); with many, one single-workgroup kernel forms it once into
// a device scalar, and the consumers read that: the bits are the same either way.  No
// atomics: results are reproducible run to run and between the batched and single-RHS
// solvers, whose partials are indexed by the block of sites they cover.
constexpr int kInlineChunks = 32;      // consuming workgroups total up to 32 chunks (2048 partials)
constexpr int kFinishThreads = 1024;   // the single-workgroup total kernels
constexpr int kMaxChunks = 4096;       // their limit: 262144 partials
inline bool totals_inline(int nparts) { return nparts <= 64 * kInlineChunks; }

// this workgroup's NV sums (wave trees, then the waves in order) to part[NV * idx + j]
template <int NT, int NV>
__device__ __forceinline__ void partials_store_at(const double (&v)[NV], double *part, int idx)
{
    __shared__ double sh[NV][NT / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; j++) {
        double s = v[j];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
        if (lane == 0) sh[j][w] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < NV; j++) {
            double b = 0;
            for (int k = 0; k < NT / 64; k++) b += sh[j][k];
            part[NV * idx + j] = b;
        }
}

// partials of an operator launch, indexed by the logical block (the sites it covers)
template <int NT, int NV>
__device__ __forceinline__ void op_partials_store(const double (&v)[NV], double *part)
{
    partials_store_at<NT, NV>(v, part, xcd_block());
}

// the total of n partials (NV interleaved values) in the fixed order above, in every thread
// of the workgroup (NT >= 128 threads, all of which must call this); at most 64 * MAXC
// partials
template <int NT, int NV, int MAXC>
__device__ __forceinline__ void partials_total(const double *__restrict__ part, int n, double (&tot)[NV])
{
    static_assert(NT >= 128 && NT % 64 == 0, "at least two waves");
    __shared__ double shc[MAXC];
    __shared__ double sh2[2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nch = (n + 63) >> 6;
    constexpr int NW = NT / 64, B = 8;   // chunks per wave and batch: their loads are issued together
#pragma unroll
    for (int j = 0; j < NV; j++) {
        for (int c0 = w; c0 < nch; c0 += NW * B) {
            double s[B];
#pragma unroll
            for (int b = 0; b < B; b++) {
                const int k = 64 * (c0 + b * NW) + lane;
                s[b] = k < n ? part[NV * k + j] : 0.0;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1)
#pragma unroll
                for (int b = 0; b < B; b++) s[b] += __shfl_down(s[b], o, 64);
            if (lane == 0)
#pragma unroll
                for (int b = 0; b < B; b++)
                    if (c0 + b * NW < nch) shc[c0 + b * NW] = s[b];
        }
        __syncthreads();
        if (threadIdx.x < 128) {
            double s = 0;
            for (int c = threadIdx.x; c < nch; c += 128) s += shc[c];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
            if (lane == 0) sh2[w] = s;
        }
        __syncthreads();
        tot[j] = sh2[0] + sh2[1];
        __syncthreads();
    }
}

// out[j] = total of n partials (one workgroup of kFinishThreads); skipped while *stop != 0
template <int NV>
__global__ __launch_bounds__(kFinishThreads) void k_total(const double *__restrict__ part, int n,
                                                         double *__restrict__ out, const double *__restrict__ stop)
{
    if (stop && stop[0] != 0) return;
    double t[NV];
    partials_total<kFinishThreads, NV, kMaxChunks>(part, n, t);
    if (threadIdx.x == 0)
        for (int j = 0; j < NV; j++) out[j] = t[j];
}

// launch k_total: the NV totals of n partials into the device scalars out (stream order)
template <int NV>
inline int launch_total(pfmp_ctx *ctx, const double *part, int n, double *out, const double *stop)
{
    if ((n + 63) / 64 > kMaxChunks) return set_err(ctx, PFMP_ERR_ARG, "totals: too many partials");
    hipLaunchKernelGGL(k_total<NV>, dim3(1), dim3(kFinishThreads), 0, ctx->stream, part, n, out, stop);
    LAUNCHCHK(ctx);
    return 0;
}


// operator stages (dslash.hip); In / X / T / Out: const C* / C* or HalfField; UL: const C*
// or HalfLinks; CL: const R* or HalfClover
template <typename C, typename R, typename In, typename Out, typename UL, typename CL>
int launch_clovinv(pfmp_ctx *ctx, int pout, In in, UL U, CL cl, Out out, R gin, R gout, bool clov,
                   const double *stop);
template <typename C, typename R, typename X, typename T, typename Out, typename UL, typename CL>
int launch_xpay(pfmp_ctx *ctx, int pout, X x, T t, UL U, CL cl, R a, Out out, R gs, bool clov, double *partials,
                const double *stop);

inline int clovinv64(pfmp_ctx *ctx, int pout, const double2 *in, const double *cl, double2 *out, double gin,
                     double gout, bool clov, const double *stop)
{
    return launch_clovinv<double2, double, const double2 *, double2 *, const double2 *, const double *>(ctx, pout, in, ctx->U, cl, out, gin, gout,
                                                                       clov, stop);
}
inline int xpay64(pfmp_ctx *ctx, int pout, const double2 *x, const double2 *t, const double *cl, double a,
                  double2 *out, double gs, bool clov, double *partials, const double *stop)
{
    return launch_xpay<double2, double, const double2 *, const double2 *, double2 *, const double2 *, const double *>(ctx, pout, x, t, ctx->U, cl, a,
                                                                                     out, gs, clov, partials, stop);
}
inline int clovinv32(pfmp_ctx *ctx, int pout, const float2 *in, const float *cl, float2 *out, float gin, float gout,
                     bool clov, const double *stop)
{
    return launch_clovinv<float2, float, const float2 *, float2 *, const float2 *, const float *>(ctx, pout, in, ctx->Uf, cl, out, gin, gout, clov,
                                                                   stop);
}
inline int xpay32(pfmp_ctx *ctx, int pout, const float2 *x, const float2 *t, const float *cl, float a, float2 *out,
                  float gs, bool clov, double *partials, const double *stop)
{
    return launch_xpay<float2, float, const float2 *, const float2 *, float2 *, const float2 *, const float *>(ctx, pout, x, t, ctx->Uf, cl, a, out,
                                                                                gs, clov, partials, stop);
}
