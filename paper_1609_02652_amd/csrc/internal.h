// internal.h -- shared device helpers and the context of libpfmp (gfx950).
//
// Internal layouts (structure of arrays, site index fastest, so that the 64 lanes
// of a wavefront read consecutive sites):
//   spinor (one parity)   c[12][Vh]           complex, component k = spin*3 + colour
//   gauge                 U[2][4][9][Vh]      complex, [parity][mu][row*3+col][eo site]
//   clover (one parity)   d[2][6][Vh] real + o[2][15][Vh] complex: the two 6x6
//                         Hermitian chiral blocks (spins {0,1} and {2,3}), diagonal
//                         and upper triangle (row-major i<j)
//   momenta / forces      P[2][4][8][Vh]      real, coefficients of T_a
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "pfmp.h"

#define PFMP_HD __host__ __device__ __forceinline__

// ------------------------------------------------------------------ complex

template <typename R> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };

template <typename C> PFMP_HD C mk(decltype(C::x) a, decltype(C::x) b) { C c; c.x = a; c.y = b; return c; }
template <typename C> PFMP_HD C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> PFMP_HD C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> PFMP_HD C cconj(C a) { return mk<C>(a.x, -a.y); }
template <typename C> PFMP_HD C cscale(C a, decltype(C::x) s) { return mk<C>(a.x * s, a.y * s); }
template <typename C> PFMP_HD C ctimesi(C a) { return mk<C>(-a.y, a.x); }     // i a
template <typename C> PFMP_HD C ctimesmi(C a) { return mk<C>(a.y, -a.x); }    // -i a
template <typename C> PFMP_HD C cneg(C a) { return mk<C>(-a.x, -a.y); }
// fused multiply-add a b + c (one rounding)
PFMP_HD double fmadd(double a, double b, double c) { return fma(a, b, c); }
PFMP_HD float fmadd(float a, float b, float c) { return fmaf(a, b, c); }
// a b and conj(a) b, each part one product and one fused multiply-add in a fixed order
// (left free, the compiler may fuse either product, and not always the same one in two
// instantiations of a kernel)
template <typename C> PFMP_HD C cmul(C a, C b)
{
    return mk<C>(fmadd(a.x, b.x, -(a.y * b.y)), fmadd(a.x, b.y, a.y * b.x));
}
template <typename C> PFMP_HD C cmulc(C a, C b)
{
    return mk<C>(fmadd(a.x, b.x, a.y * b.y), fmadd(a.x, b.y, -(a.y * b.x)));
}
// s += |v|^2 in FP64, in a fixed order
template <typename C> PFMP_HD void cnorm_acc(double &s, C v)
{
    s = fmadd((double)v.y, (double)v.y, fmadd((double)v.x, (double)v.x, s));
}
// acc += a * b as four fused multiply-adds
template <typename C> PFMP_HD void cfma(C &acc, C a, C b)
{
    acc.x = fmadd(-a.y, b.y, fmadd(a.x, b.x, acc.x));
    acc.y = fmadd(a.y, b.x, fmadd(a.x, b.y, acc.y));
}
// acc += conj(a) * b
template <typename C> PFMP_HD void cfmac(C &acc, C a, C b)
{
    acc.x = fmadd(a.y, b.y, fmadd(a.x, b.x, acc.x));
    acc.y = fmadd(-a.y, b.x, fmadd(a.x, b.y, acc.y));
}

// ------------------------------------------------------------------ geometry

struct Geom {
    int L[4];
    int Lh0;        // Lx / 2
    int Vh;
    int V;
    int tbc;        // fermion factor across the t boundary
    int recon;      // 1: every link is in SU(3), the hopping kernels rebuild row 3 from rows 1, 2
    int zt;         // site visit order of the operator kernels: 0 natural, else groups of zt z-planes
    int stream;     // 1: the hopping kernels load links with streaming (non-temporal) loads
};

// link mode of the hopping kernels: bit 0 row reconstruction, bit 1 streaming loads
inline int link_mode(const Geom &g) { return (g.recon ? 1 : 0) | (g.stream ? 2 : 0); }
#define PFMP_LM_SWITCH(lm, M)        \
    switch (lm) {                    \
    case 0: M(0); break;             \
    case 1: M(1); break;             \
    case 2: M(2); break;             \
    default: M(3); break;            \
    }

// Coordinates of even-odd site i of parity p: lex = 2i or 2i+1, whichever has parity p.
__device__ __forceinline__ void eo_coords(const Geom &g, int p, int i, int c[4])
{
    int r = i / g.Lh0;
    int xh = i - r * g.Lh0;
    int y = r % g.L[1];
    int r2 = r / g.L[1];
    int z = r2 % g.L[2];
    int t = r2 / g.L[2];
    c[0] = 2 * xh + ((p + y + z + t) & 1);
    c[1] = y;
    c[2] = z;
    c[3] = t;
}

// Even-odd index of the site with coordinates c (its parity is implied).
__device__ __forceinline__ int eo_index(const Geom &g, const int c[4])
{
    return (c[0] >> 1) + g.Lh0 * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}

// Even-odd index of the neighbour of site c in direction mu, step +1 / -1, and
// the fermion boundary factor of that hop.
__device__ __forceinline__ int eo_neighbour(const Geom &g, const int c[4], int mu, int step, int *fsign)
{
    int d[4] = {c[0], c[1], c[2], c[3]};
    int v = d[mu] + step;
    int s = 1;
    if (v == g.L[mu]) { v = 0; if (mu == 3) s = g.tbc; }
    if (v < 0) { v = g.L[mu] - 1; if (mu == 3) s = g.tbc; }
    d[mu] = v;
    *fsign = s;
    return eo_index(g, d);
}

// Even-odd index of the l-th site in the visit order of the operator kernels.  With
// zt > 0 the (x, y) planes are visited in memory order, zt z-planes at a time, then the
// next t, and only then the next group of z-planes: the spinors of the t - 1, t, t + 1
// slices of one group stay in L2 until their last use instead of a whole 3 t-slices.
__device__ __forceinline__ int tile_site(const Geom &g, int l)
{
    if (g.zt <= 0) return l;
    const int plane = g.Lh0 * g.L[1];
    const int xy = l % plane;
    int r = l / plane;
    const int zi = r % g.zt;
    r /= g.zt;
    const int t = r % g.L[3], zb = r / g.L[3];
    return xy + plane * (zb * g.zt + zi + g.L[2] * t);
}

// Site of this thread with an XCD-aware block order: the hardware hands
// consecutive workgroups round-robin to the 8 XCDs (each with its own L2), so
// logical block b' = (b mod 8) * ceil(nb/8) + b / 8 gives every XCD one
// contiguous chunk of sites and keeps the y, z, t neighbour gathers in its L2.
// Returns -1 for threads past the end.
__device__ __forceinline__ int xcd_site(int n)
{
    const int nb = gridDim.x, b = blockIdx.x;
    const int per = (nb + 7) >> 3;
    const int lb = (b & 7) * per + (b >> 3);
    if (lb >= nb) return -1;
    int i = lb * blockDim.x + threadIdx.x;
    return i < n ? i : -1;
}

// Logical block of this workgroup in the order above (a bijection onto [0, nb) when the
// grid is a multiple of 8 workgroups, as for every operator launch)
__device__ __forceinline__ int xcd_block()
{
    const int nb = gridDim.x, b = blockIdx.x;
    const int per = (nb + 7) >> 3;
    return (b & 7) * per + (b >> 3);
}

// The same block order for kernels with more lanes than the int range may hold
// (several lanes per link or plane): the lane index, or n for every lane of the
// blocks past the end, so that the kernel's own bound check (lane < n) drops them.
__device__ __forceinline__ long xcd_lane(long n)
{
    const int nb = gridDim.x, b = blockIdx.x;
    const int per = (nb + 7) >> 3;
    const int lb = (b & 7) * per + (b >> 3);
    return lb < nb ? (long)lb * blockDim.x + threadIdx.x : n;
}

// ------------------------------------------------------------------ context

struct OpSlot {
    bool valid = false;
    double kappa = 0, csw = 0;
    double *clov[2] = {nullptr, nullptr};   // FP64: A_ee on [0] (even), A_oo^-1 on [1] (odd)
    float *clovf[2] = {nullptr, nullptr};   // FP32 copies
    void *clovh[2] = {nullptr, nullptr};    // FP16 copies (binary16 reals, same layout)
    double logdet_odd = 0;                  // sum_{x odd} ln det A(x)
    double *ldpart = nullptr;               // per-block ln det A_oo partials (device)
    bool ld_dirty = false;                  // ldpart newer than logdet_odd
    bool stale = false;                     // links changed since the clover fields were built
};

struct SolverWS;

struct pfmp_ctx {
    Geom g;
    hipStream_t stream = nullptr;
    int nblk_red = 0;            // blocks of the reduction kernels
    double2 *U = nullptr;        // internal FP64 gauge field
    float2 *Uf = nullptr;        // FP32 copy
    void *Uh = nullptr;          // FP16 copy (binary16 complex planes), for the FP16-storage inner solver
    bool have_gauge = false;
    bool uf_stale = true;        // Uf older than U
    double2 *Fhat = nullptr;     // clover field strength [2 parities][6 planes][9][Vh], shared by all slots
    bool fhat_stale = true;      // Fhat older than U
    bool recon_allowed = true;   // link row reconstruction permitted (pfmp_set_link_reconstruct)
    bool links_su3 = false;      // the links passed the SU(3) check at set_gauge
    OpSlot ops[PFMP_MAX_OPS];
    double *red = nullptr;       // reduction partials
    double *red_host = nullptr;  // pinned host mirror of a few scalars
    double *scal = nullptr;      // device scalars for solvers
    void *scratch = nullptr;     // this GPU's static scratch of pfmp_apply_MdagM_noalloc (device address)
    SolverWS *ws = nullptr;
    std::vector<double2 *> pool;   // FP64 spinor buffers for the HMC driver, grown on demand
    bool use_graphs = true;        // solver iterations replayed as HIP graphs
    bool half_links = true;        // FP16-storage solver reads the FP16 copies of links and clover
    int verbose = 0;               // 1: the HMC driver prints its progress to stderr
    int batch_multi = 1;           // batched clover stencils: 0 one workgroup per (site block, rhs); 1 the
                                   // default group of rhs per lane pair sharing link loads; 2 or 4 that group
    // clover-force insertions of several force terms summed into one field before a single
    // clover-force pass (set by the integrator for the terms due at one merged step)
    bool clover_defer = false;
    bool phi_pending = false;      // the insertion field holds terms not yet applied
    hipStream_t cap = nullptr;     // private stream the graphs are captured on
    struct Graph {
        std::vector<uint64_t> key;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;     // captured iterations, most recent last
    std::string err;
};

// ------------------------------------------------------------------ errors

int set_err(pfmp_ctx *ctx, int code, const std::string &msg);

#define HIPCHK(ctx, call)                                                                            \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return set_err((ctx), PFMP_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

#define LAUNCHCHK(ctx)                                                                                   \
    do {                                                                                                 \
        hipError_t e_ = hipGetLastError();                                                               \
        if (e_ != hipSuccess)                                                                            \
            return set_err((ctx), PFMP_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------ launch sizes

constexpr int kBlock = 128;      // threads per block of the site kernels
constexpr int kRedBlock = 256;   // threads per block of reductions
inline int nblocks(long n, int b) { return (int)((n + b - 1) / b); }
// grid of the site kernels that use xcd_site(): a multiple of 8 blocks so that the
// XCD block order is a bijection
inline int nblocks_site(long n) { return ((nblocks(n, kBlock) + 7) / 8) * 8; }

// sizes of internal fields
inline long spinor_reals(const Geom &g) { return 24L * g.Vh; }
// grid of the operator kernels (two lanes per site) = number of block partials they write
inline int op_nparts(const Geom &g) { return nblocks_site(2L * g.Vh); }
inline long clover_reals(const Geom &g) { return 72L * g.Vh; }
inline long gauge_reals(const Geom &g) { return 2L * 4 * 18 * g.Vh; }
inline long mom_reals(const Geom &g) { return 2L * 4 * 8 * g.Vh; }

// ------------------------------------------------------------------ internal API

// operator stages (dslash.hip)
int op_apply_M(pfmp_ctx *ctx, int op, int dagger, const double2 *in, double2 *out, double2 *tmp_odd,
               double *norm_partials);
int op_apply_K(pfmp_ctx *ctx, int op, const double2 *in, double2 *out, double2 *tmp_even, double2 *tmp_odd,
               double *norm_partials);
int op_apply_M_f32(pfmp_ctx *ctx, int op, int dagger, const float2 *in, float2 *out, float2 *tmp_odd,
                   double *norm_partials);
int op_apply_K_f32(pfmp_ctx *ctx, int op, const float2 *in, float2 *out, float2 *tmp_even, float2 *tmp_odd,
                   double *norm_partials);
int rebuild_gauge_derived(pfmp_ctx *ctx);
int red_finish_dev(pfmp_ctx *ctx, const double *partials, int nparts, int nvals, double *dev_out);
// clover (clover.hip)
int clover_build(pfmp_ctx *ctx, int op);
// slot valid and its clover fields current (rebuilt on first use after a link update)
int op_ready(pfmp_ctx *ctx, int op);
// FP32 copy of the links current (context.hip)
int gauge_f32_ready(pfmp_ctx *ctx);
// Launch `issue` (a fixed sequence of kernel launches on ctx->stream) reps times.  With
// graphs on, the sequence is captured once as a HIP graph under `key` (every pointer and
// value its launches use) and replayed; otherwise it is issued reps times.
int graph_run(pfmp_ctx *ctx, const std::vector<uint64_t> &key, int reps, const std::function<int()> &issue);
template <typename T>
inline void key_add(std::vector<uint64_t> &k, const T &v)
{
    static_assert(sizeof(T) <= 8, "key entries are at most 8 bytes");
    uint64_t u = 0;
    std::memcpy(&u, &v, sizeof(T));
    k.push_back(u);
}
inline void key_geom(std::vector<uint64_t> &k, const Geom &g)
{
    for (int m = 0; m < 4; m++) key_add(k, g.L[m]);
    key_add(k, g.tbc);
    key_add(k, g.recon);
    key_add(k, g.zt);
    key_add(k, g.stream);
}
int clover_logdet(pfmp_ctx *ctx, int op);
// force.hip: start collecting clover insertions; apply what was collected (F += its force)
void clover_force_defer(pfmp_ctx *ctx);
int clover_force_flush(pfmp_ctx *ctx, double *F);
// maximum and mean over links of the force norm (sum_a F_a^2)^(1/2); synchronises
int force_norms(pfmp_ctx *ctx, const double *F, double *mx, double *mean);
// pfmp_fermion_force with FP32 spinors (intermediates by the FP32 operator, force in FP64)
int fermion_force_f32(pfmp_ctx *ctx, int op, int npairs, const void *const *X, const void *const *Y,
                      const double *coeff, double *F);
// reductions (blas.hip)
int red_finish(pfmp_ctx *ctx, const double *partials, int nparts, int nvals, double *host_out);
int launch_dot(pfmp_ctx *ctx, const double2 *a, const double2 *b, long n, double *partials);
int launch_norm2(pfmp_ctx *ctx, const double2 *a, long n, double *partials);
void *ws_alloc(pfmp_ctx *ctx, size_t bytes, int slot);
double2 *pool_get(pfmp_ctx *ctx, int idx);
// polynomial (poly.hip)
int poly_factor(pfmp_ctx *ctx, int op, const double2 *src, double2 z, double2 *dst, double2 *te, double2 *to);
int scale_spinor(pfmp_ctx *ctx, double2 a, const double2 *x, double2 *y);
// device address of the allocation-free entry point's static scratch on the current GPU
// (dslash.hip), looked up once per device; called at context creation
int noalloc_scratch_init(pfmp_ctx *ctx);
// mixed precision (mixed.hip)
int cg_solve_mixed(pfmp_ctx *ctx, int op, const void *b, void *x, const pfmp_solver_params *p,
                   pfmp_solver_stats *st);
