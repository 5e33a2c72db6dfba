// force.hip -- molecular-dynamics forces (paper App. C) and the atomic
// integrator steps T and S (App. B, eq. time_update / space_update).
//
// Forces are Lie-algebra coefficients f_a = d/dw S along U -> exp(i w T_a) U.  For
// every link the kernels build a 3x3 matrix Z with f_a = Re tr[i T_a Z].
//
// Fermion bilinear Re[c X^dag Mhat Y], Mhat = A_ee - kappa^2 D_eo A_oo^-1 D_oe:
// with L = (X | Xo) and R = (Y | Z) on (even | odd) sites, Xo = A_oo^-1 (D_eo)^dag X,
// Z = A_oo^-1 D_oe Y, the derivative is
//   sum_x L^dag [ w(x) dA(x) R - kappa^2 (dD_hop R)(x) ],  w = 1 (even), kappa^2 (odd).
// Hopping part, link U = U_mu(x) between x and x+mu with boundary factor s:
//   Z_hop = c s (U G_A - G_B U^dag),
//   G_A = sum_t g_t h_t^dag with g, h the (1 - g_mu) half spinors of R(x+mu), L(x),
//   G_B = the same with (1 + g_mu) half spinors of R(x), L(x+mu).
// Clover part: per site and plane p the colour matrix
//   Phi_p(x) = c w i kappa c_sw sum_{s,t} sigma_p[s][t] R_t L_s^dag
// (log-det term: -2 i kappa c_sw sum sigma_p[s][t] (A^-1)_{t s} on odd sites) so that
// the contribution is Re tr[dFhat_p Phi_p] = Re tr[dQ_p Psi_p], Psi_p = (Phi_p - Phi_p^dag)/8;
// each link then collects, over the 2 plaquettes x 4 corners of every plane holding
// it, the leaf products with Psi inserted at the corner.
#include <type_traits>
#include <vector>

#include "hop.h"
#include "su3.h"

namespace {

// chiral-block Pauli structure of sigma_p: type (0 = x, 1 = y, 2 = z) and signs on
// the upper / lower block; plane order (01)(02)(03)(12)(13)(23)
__constant__ int kSigType[6] = {2, 1, 0, 0, 1, 2};
__constant__ double kSigUp[6] = {-1, 1, 1, -1, 1, 1};
__constant__ double kSigLo[6] = {-1, 1, -1, -1, -1, -1};

// sum_{s,t} pauli[s][t] O_{st} for O_{st} given as 4 matrices O[2*s+t]
__device__ __forceinline__ M3 pauli_contract(int type, const M3 *O)
{
    if (type == 0) return m3_add(O[1], O[2]);                                    // s_x
    if (type == 1) {                                                             // s_y: -i O01 + i O10
        M3 r;
        for (int k = 0; k < 9; k++) r.e[k] = csub(ctimesi(O[2].e[k]), ctimesi(O[1].e[k]));
        return r;
    }
    return m3_sub(O[0], O[3]);                                                   // s_z
}

// ---------------------------------------------------------------- hop part

// Up to kForcePairs bilinears (X_q, Y_q) with coefficients c_q in one launch; Xo_q and
// Zo_q are their odd-site intermediates (see the header).
// The spinors are FP64 (C = double2) or FP32 (float2, widened on load); the force is
// accumulated in FP64 either way.
constexpr int kForcePairs = 8;
template <typename C>
struct PairSet {
    int n;
    const C *X[kForcePairs], *Xo[kForcePairs], *Y[kForcePairs], *Zo[kForcePairs];
    double2 c[kForcePairs];
};

// the 12 components of a spinor at site i, in FP64
template <typename C>
__device__ __forceinline__ void load_wide(const C *__restrict__ f, int Vh, int i, double2 *v)
{
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const C a = f[(long)k * Vh + i];
        v[k] = make_double2((double)a.x, (double)a.y);
    }
}

// c (U G_A) + conj(c) (U G_B^dag): the coefficient map is odd under Z -> Z^dag, so
// this gives the force of c (U G_A - G_B U^dag)
template <int MU, typename C>
__device__ __forceinline__ void hop_force_link(const Geom &g, int p, int i, const int *c, const PairSet<C> &ps,
                                               const double2 *__restrict__ U, double scale, double *__restrict__ F)
{
    int s;
    const int j = eo_neighbour(g, c, MU, +1, &s);
    M3 M = m3_zero();
    for (int q = 0; q < ps.n; q++) {
        const C *Lx = p == 0 ? ps.X[q] : ps.Xo[q], *Rx = p == 0 ? ps.Y[q] : ps.Zo[q];
        const C *Ly = p == 0 ? ps.Xo[q] : ps.X[q], *Ry = p == 0 ? ps.Zo[q] : ps.Y[q];
        double2 v[12], hL[6], hR[6];
        // G_A: (1 - g) projections of R(x+mu) and L(x)
        load_wide(Ry, g.Vh, j, v);
        project<MU, -1>(v, hR);
        load_wide(Lx, g.Vh, i, v);
        project<MU, -1>(v, hL);
        const double2 cq = ps.c[q], cc = cconj(cq);
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                double2 o = cadd(cmulc(hL[b], hR[a]), cmulc(hL[3 + b], hR[3 + a]));   // (G_A)_ab
                cfma(M.e[3 * a + b], cq, o);
            }
        // G_B: (1 + g) projections of R(x) and L(x+mu); add conj(c) G_B^dag
        load_wide(Rx, g.Vh, i, v);
        project<MU, +1>(v, hR);
        load_wide(Ly, g.Vh, j, v);
        project<MU, +1>(v, hL);
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                double2 o = cadd(cmulc(hL[b], hR[a]), cmulc(hL[3 + b], hR[3 + a]));   // (G_B)_ab
                cfma(M.e[3 * b + a], cc, cconj(o));
            }
    }
    M3 Uu;
    const double2 *ub = U + ((long)(p * 4 + MU) * 9) * g.Vh + i;
#pragma unroll
    for (int k = 0; k < 9; k++) Uu.e[k] = ub[(long)k * g.Vh];
    double f[8];
    lie_coeffs(m3_mul(Uu, M), f);
    double *fb = F + ((long)(p * 4 + MU) * 8) * g.Vh + i;
    const double sc = scale * (double)s;
#pragma unroll
    for (int a = 0; a < 8; a++) fb[(long)a * g.Vh] += sc * f[a];
}

// F[link] += scale * (hopping-term force of all pairs); one thread per link
template <typename C>
__global__ __launch_bounds__(kBlock) void k_hop_force_multi(Geom g, PairSet<C> ps, const double2 *__restrict__ U,
                                                            double scale, double *__restrict__ F)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= 8L * g.Vh) return;
    const int mu = (int)(t / (2L * g.Vh));
    const long r = t - (long)mu * 2L * g.Vh;
    const int p = (int)(r / g.Vh), i = (int)(r - (long)p * g.Vh);
    int c[4];
    eo_coords(g, p, i, c);
    switch (mu) {
    case 0: hop_force_link<0>(g, p, i, c, ps, U, scale, F); break;
    case 1: hop_force_link<1>(g, p, i, c, ps, U, scale, F); break;
    case 2: hop_force_link<2>(g, p, i, c, ps, U, scale, F); break;
    default: hop_force_link<3>(g, p, i, c, ps, U, scale, F); break;
    }
}

// Phi_pl(x) (+)= sum_q fac(x) c_q sum_{s,t} sigma_pl[s][t] R_t L_s^dag, fac = fe (even) / fo
// (odd), L = (X | Xo), R = (Y | Zo); one thread per (parity, plane, site)
template <typename C>
__global__ __launch_bounds__(kBlock) void k_clover_insert_multi(Geom g, PairSet<C> ps, double2 fe, double2 fo,
                                                                int accumulate, double2 *__restrict__ Phi)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= 12L * g.Vh) return;
    const int pp = (int)(t / g.Vh), i = (int)(t - (long)pp * g.Vh);
    const int p = pp / 6, pl = pp - 6 * p;
    const int type = kSigType[pl];
    const double su = kSigUp[pl], sl = kSigLo[pl];
    M3 acc = m3_zero();
    for (int q = 0; q < ps.n; q++) {
        const C *L = p == 0 ? ps.X[q] : ps.Xo[q], *R = p == 0 ? ps.Y[q] : ps.Zo[q];
        const double2 cq = cmul(ps.c[q], p == 0 ? fe : fo);
#pragma unroll
        for (int blk = 0; blk < 2; blk++) {
            double2 r0[3], r1[3], l0[3], l1[3];
#pragma unroll
            for (int a = 0; a < 3; a++) {
                const C ra = R[(long)(6 * blk + a) * g.Vh + i], rb = R[(long)(6 * blk + 3 + a) * g.Vh + i];
                const C la = L[(long)(6 * blk + a) * g.Vh + i], lb = L[(long)(6 * blk + 3 + a) * g.Vh + i];
                r0[a] = make_double2((double)ra.x, (double)ra.y);
                r1[a] = make_double2((double)rb.x, (double)rb.y);
                l0[a] = make_double2((double)la.x, (double)la.y);
                l1[a] = make_double2((double)lb.x, (double)lb.y);
            }
            const double2 w = cscale(cq, blk ? sl : su);
#pragma unroll
            for (int a = 0; a < 3; a++)
#pragma unroll
                for (int b = 0; b < 3; b++) {
                    double2 o;
                    if (type == 0) o = cadd(cmulc(l0[b], r1[a]), cmulc(l1[b], r0[a]));                 // s_x
                    else if (type == 1) o = ctimesi(csub(cmulc(l1[b], r0[a]), cmulc(l0[b], r1[a])));   // s_y
                    else o = csub(cmulc(l0[b], r0[a]), cmulc(l1[b], r1[a]));                           // s_z
                    cfma(acc.e[3 * a + b], w, o);
                }
        }
    }
    double2 *o = Phi + ((long)pp * 9) * g.Vh + i;
#pragma unroll
    for (int k = 0; k < 9; k++) o[(long)k * g.Vh] = accumulate ? cadd(o[(long)k * g.Vh], acc.e[k]) : acc.e[k];
}

// ---------------------------------------------------------------- clover insertions

// Phi[site][plane] layout: ((p * 6 + plane) * 9 + k) * Vh + i  (complex)
__device__ __forceinline__ void phi_add(const Geom &g, double2 *__restrict__ Phi, int p, int i, int plane, const M3 &m)
{
    double2 *b = Phi + ((long)(p * 6 + plane) * 9) * g.Vh + i;
    for (int k = 0; k < 9; k++) b[(long)k * g.Vh] = cadd(b[(long)k * g.Vh], m.e[k]);
}

// Phi_p(x) += fac * sum_{s,t} sigma_p[s][t] (A^-1)_{(t),(s)} on odd sites (log-det term)
__global__ __launch_bounds__(kBlock) void k_logdet_insert(Geom g, const double *__restrict__ cl, double2 fac,
                                                          double2 *__restrict__ Phi)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.Vh) return;
    const double2 *off = reinterpret_cast<const double2 *>(cl + 12L * g.Vh);
    M3 O[2][4];
    for (int b = 0; b < 2; b++) {
        double2 A[36];
        int m = 0;
        for (int r = 0; r < 6; r++) {
            A[r * 6 + r] = make_double2(cl[(long)(b * 6 + r) * g.Vh + i], 0);
            for (int q = r + 1; q < 6; q++, m++) {
                double2 v = off[(long)(b * 15 + m) * g.Vh + i];
                A[r * 6 + q] = v;
                A[q * 6 + r] = cconj(v);
            }
        }
        // O[s*2+t] = colour block (t, s) of A^-1 within the chiral block
        for (int s = 0; s < 2; s++)
            for (int t = 0; t < 2; t++)
                for (int a = 0; a < 3; a++)
                    for (int bb = 0; bb < 3; bb++) O[b][2 * s + t].e[3 * a + bb] = A[(3 * t + a) * 6 + 3 * s + bb];
    }
    for (int pl = 0; pl < 6; pl++) {
        M3 a = m3_scale(pauli_contract(kSigType[pl], O[0]), kSigUp[pl]);
        M3 b = m3_scale(pauli_contract(kSigType[pl], O[1]), kSigLo[pl]);
        phi_add(g, Phi, 1, i, pl, m3_cscale(m3_add(a, b), fac));
    }
}

// Psi = (Phi - Phi^dag) / 8 per parity, plane and site, packed as the 9 reals of an
// anti-Hermitian 3x3 matrix: Im of the 3 diagonal entries, then Re, Im of entries
// (0,1), (0,2), (1,2); layout ((p * 6 + plane) * 9 + k) * Vh + i.  Built once per
// force evaluation, it halves (and packs) what the clover force reads per insertion.
constexpr int kPsiReals = 9;

__global__ void k_psi_pack(Geom g, const double2 *__restrict__ Phi, double *__restrict__ Psi)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= 12L * g.Vh) return;
    const long pp = t / g.Vh, i = t - pp * g.Vh;   // pp = parity * 6 + plane
    const double2 *b = Phi + pp * 9 * g.Vh + i;
    double *o = Psi + pp * kPsiReals * g.Vh + i;
    const long st = g.Vh;
#pragma unroll
    for (int d = 0; d < 3; d++) o[d * st] = 0.25 * b[(4 * d) * st].y;   // (Phi - Phi^*)_dd / 8 = i Im / 4
    const int rc[3][2] = {{0, 1}, {0, 2}, {1, 2}};
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const double2 u = b[(3 * rc[q][0] + rc[q][1]) * st], l = b[(3 * rc[q][1] + rc[q][0]) * st];
        o[(3 + 2 * q) * st] = 0.125 * (u.x - l.x);       // Re (Phi_rc - conj Phi_cr) / 8
        o[(4 + 2 * q) * st] = 0.125 * (u.y + l.y);       // Im
    }
}

// Psi_mu_nu at the site with coordinates c as a 3x3 matrix, Psi_nu_mu = -Psi_mu_nu
__device__ __forceinline__ M3 psi_at(const Geom &g, const double *__restrict__ Psi, const int *c, int mu, int nu)
{
    const int p = parity_of(c), i = eo_index(g, c);
    const int a = mu < nu ? mu : nu, bb = mu < nu ? nu : mu;
    const double sc = mu < nu ? 1.0 : -1.0;
    const double *b = Psi + ((long)(p * 6 + plane_index(a, bb)) * kPsiReals) * g.Vh + i;
    const long st = g.Vh;
    double v[kPsiReals];
#pragma unroll
    for (int k = 0; k < kPsiReals; k++) v[k] = sc * b[k * st];
    M3 r;
    r.e[0] = make_double2(0, v[0]);
    r.e[4] = make_double2(0, v[1]);
    r.e[8] = make_double2(0, v[2]);
    r.e[1] = make_double2(v[3], v[4]);
    r.e[3] = make_double2(-v[3], v[4]);   // Psi_10 = -conj(Psi_01)
    r.e[2] = make_double2(v[5], v[6]);
    r.e[6] = make_double2(-v[5], v[6]);
    r.e[5] = make_double2(v[7], v[8]);
    r.e[7] = make_double2(-v[7], v[8]);
    return r;
}

// Clover force: F[link] += coefficients of U_mu(y) S with
//   S = sum_{nu != mu} sum_{s = +1, -1} s * sum over the 4 corners of the leaf that
//       runs y+mu -> y+mu+s nu -> y+s nu -> y of the path with Psi inserted at the corner.
// The leaf below the link enters as the adjoint of its own path: the coefficient map
// Z -> Re tr[i T_a Z] is odd under Z -> Z^dag and Psi is anti-Hermitian, so
// -W_b U^dag and U W_b^dag give the same force.  With the path L1 L2 L3 and corner
// insertions Psi1..Psi4 the sum is taken Horner-fashion:
//   Q = Psi1 L1 + L1 Psi2,  Q = Q L2 + (L1 L2) Psi3,  Q = Q L3 + (L1 L2 L3) Psi4.
// Two lanes per link (the two sides s); the 8 coefficients of each leaf are
// accumulated and the two lanes summed by a lane swap.
__global__ __launch_bounds__(kBlock) void k_clover_force(Geom g, const double2 *__restrict__ U,
                                                         const double *__restrict__ Psi, double *__restrict__ F)
{
    const long t = xcd_lane(16L * g.Vh);   // XCD-aware order, as the gauge force
    const long l = t >> 1;
    const int side = (int)(t & 1);
    const bool ok = l < 8L * g.Vh;
    double f[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int mu = 0, p = 0, i = 0;
    if (ok) {
        mu = (int)(l / (2L * g.Vh));
        const long r = l - (long)mu * 2L * g.Vh;
        p = (int)(r / g.Vh);
        i = (int)(r - (long)p * g.Vh);
        int y[4], ypm[4];
        eo_coords(g, p, i, y);
        shifted(g, y, mu, +1, ypm);
        const int sg = side ? -1 : 1;
#pragma unroll 1
        for (int nu = 0; nu < 4; nu++) {
            if (nu == mu) continue;
            int yn[4], ypmn[4];
            shifted(g, y, nu, sg, yn);          // y + s nu
            shifted(g, ypm, nu, sg, ypmn);      // y + mu + s nu
            // L1: y+mu -> y+mu+s nu
            M3 L1 = m3_dag_if(link_at(g, U, side ? ypmn : ypm, nu), side);
            M3 Q = m3_mul(psi_at(g, Psi, ypm, mu, nu), L1);
            Q = m3_add(Q, m3_mul(L1, psi_at(g, Psi, ypmn, mu, nu)));
            // L2: y+mu+s nu -> y+s nu
            M3 L2 = m3_dag(link_at(g, U, yn, mu));
            M3 R = m3_mul(L1, L2);
            Q = m3_mul(Q, L2);
            Q = m3_add(Q, m3_mul(R, psi_at(g, Psi, yn, mu, nu)));
            // L3: y+s nu -> y
            M3 L3 = m3_dag_if(link_at(g, U, side ? yn : y, nu), !side);
            R = m3_mul(R, L3);
            Q = m3_mul(Q, L3);
            Q = m3_add(Q, m3_mul(R, psi_at(g, Psi, y, mu, nu)));
            // coefficients of s U_mu(y) Q
            double fl[8];
            lie_coeffs(m3_mul(link_at(g, U, y, mu), Q), fl);
#pragma unroll
            for (int a = 0; a < 8; a++) f[a] += side ? -fl[a] : fl[a];
        }
    }
#pragma unroll
    for (int a = 0; a < 8; a++) f[a] += __shfl_xor(f[a], 1, 64);
    if (ok && side == 0) {
        double *fb = F + ((long)(p * 4 + mu) * 8) * g.Vh + i;
#pragma unroll
        for (int a = 0; a < 8; a++) fb[(long)a * g.Vh] += f[a];
    }
}

// ---------------------------------------------------------------- gauge part

// F[link] += coefficients of coef U_mu(y) (sum of the staples); two lanes per link, the
// staples above (lane 0) and below (lane 1) the link, coefficients summed by a lane swap
__global__ __launch_bounds__(kBlock) void k_gauge_force(Geom g, const double2 *__restrict__ U, double coef,
                                                        double *__restrict__ F)
{
    // XCD-aware order: each XCD takes a contiguous eighth of the links (one direction and
    // parity), so the staples' neighbour links are gathered through its own L2
    const long t = xcd_lane(16L * g.Vh);
    const long l = t >> 1;
    const int side = (int)(t & 1);
    const bool ok = l < 8L * g.Vh;
    double f[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int mu = 0, p = 0, i = 0;
    if (ok) {
        mu = (int)(l / (2L * g.Vh));
        const long r = l - (long)mu * 2L * g.Vh;
        p = (int)(r / g.Vh);
        i = (int)(r - (long)p * g.Vh);
        int y[4], ypm[4];
        eo_coords(g, p, i, y);
        shifted(g, y, mu, +1, ypm);
        M3 st = m3_zero();
        const int sg = side ? -1 : 1;
#pragma unroll 1
        for (int nu = 0; nu < 4; nu++) {
            if (nu == mu) continue;
            // path y+mu -> y+mu+s nu -> y+s nu -> y:
            //   s = +1: U_nu(y+mu) U_mu(y+nu)^dag U_nu(y)^dag
            //   s = -1: U_nu(y+mu-nu)^dag U_mu(y-nu)^dag U_nu(y-nu)
            int yn[4], ypmn[4];
            shifted(g, y, nu, sg, yn);
            shifted(g, ypm, nu, sg, ypmn);
            // the two nu links' sites, chosen element-wise so that the arrays stay in registers
            int a1[4], a3[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                a1[k] = side ? ypmn[k] : ypm[k];
                a3[k] = side ? yn[k] : y[k];
            }
            M3 X1 = m3_dag_if(link_at_su3(g, U, a1, nu), side);
            M3 X3 = m3_dag_if(link_at_su3(g, U, a3, nu), !side);
            st = m3_add(st, m3_mul(X1, m3_mul_dn(link_at_su3(g, U, yn, mu), X3)));
        }
        lie_coeffs(m3_scale(m3_mul(link_at_su3(g, U, y, mu), st), coef), f);
    }
#pragma unroll
    for (int a = 0; a < 8; a++) f[a] += __shfl_xor(f[a], 1, 64);
    if (ok && side == 0) {
        double *fb = F + ((long)(p * 4 + mu) * 8) * g.Vh + i;
#pragma unroll
        for (int a = 0; a < 8; a++) fb[(long)a * g.Vh] += f[a];
    }
}

// ---------------------------------------------------------------- updates

__global__ void k_update_momenta(long n, double eps, const double *__restrict__ F, double *__restrict__ P)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) P[t] -= eps * F[t];
}

// exp(Q) for anti-Hermitian traceless Q: scaling and squaring with a Taylor polynomial
// (Horner) on A = Q / 2^k, a = |A|_F <= 1/4.  The degree m is the smallest (at most 14)
// whose first dropped term a^(m+1) / (m+1)! is at most 2^-60; the whole remainder is then
// below 1.1 times that, far under the rounding of the result.  MD steps give a of order
// 0.01 and m = 7 or less; a = 1/4 needs m = 13.
__device__ M3 expm_ah(const M3 &Q)
{
    double nrm = 0;
    for (int k = 0; k < 9; k++) nrm += Q.e[k].x * Q.e[k].x + Q.e[k].y * Q.e[k].y;
    nrm = sqrt(nrm);
    int sq = 0;
    double sc = 1;
    while (nrm * sc > 0.25 && sq < 40) { sc *= 0.5; sq++; }
    const double a = nrm * sc;
    int m = 1;
    for (double term = a; m < 14 && term * a / (m + 1) > 0x1p-60; m++) term *= a / (m + 1);
    M3 A = m3_scale(Q, sc);
    M3 E = m3_eye();
    for (int k = m; k >= 1; k--) {
        E = m3_scale(m3_mul(A, E), 1.0 / k);
        E.e[0].x += 1; E.e[4].x += 1; E.e[8].x += 1;
    }
    for (int s = 0; s < sq; s++) E = m3_mul(E, E);
    return E;
}

__global__ void k_update_gauge(Geom g, double eps, const double *__restrict__ P, double2 *__restrict__ U)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= 2L * g.Vh * 4) return;
    int mu = (int)(t / (2L * g.Vh));
    long r = t % (2L * g.Vh);
    int p = (int)(r / g.Vh), i = (int)(r % g.Vh);
    double pa[8];
    const double *pb = P + ((long)(p * 4 + mu) * 8) * g.Vh + i;
    for (int a = 0; a < 8; a++) pa[a] = pb[(long)a * g.Vh];
    M3 H = lie_matrix(pa);
    M3 Q;
    for (int k = 0; k < 9; k++) Q.e[k] = cscale(ctimesi(H.e[k]), eps);   // i eps P
    M3 E = expm_ah(Q);
    double2 *ub = U + ((long)(p * 4 + mu) * 9) * g.Vh + i;
    M3 Uu;
    for (int k = 0; k < 9; k++) Uu.e[k] = ub[(long)k * g.Vh];
    M3 Un = m3_mul(E, Uu);
    for (int k = 0; k < 9; k++) ub[(long)k * g.Vh] = Un.e[k];
}

// ---------------------------------------------------------------- actions

__device__ __forceinline__ void block_partial(double v, double *out)
{
    __shared__ double sh[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
        for (int k = 0; k < kBlock / 64; k++) s += sh[k];
        out[blockIdx.x] = s;
    }
}

// sum over plaquettes of (1 - Re tr U_P / 3), one thread per site
__global__ __launch_bounds__(kBlock) void k_plaq(Geom g, const double2 *__restrict__ U, double *__restrict__ part)
{
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    double s = 0;
    if (t < 2L * g.Vh) {
        int p = (int)(t / g.Vh), i = (int)(t % g.Vh);
        int c[4];
        eo_coords(g, p, i, c);
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                int a[4], b[4];
                shifted(g, c, mu, +1, a);
                shifted(g, c, nu, +1, b);
                M3 P = m3_mul_nd(m3_mul(link_at(g, U, c, mu), link_at(g, U, a, nu)),
                                 m3_mul(link_at(g, U, c, nu), link_at(g, U, b, mu)));
                s += 1.0 - m3_trace(P).x / 3.0;
            }
    }
    block_partial(s, part);
}

// 1/2 sum_a p_a^2 = sum tr P^2
__global__ __launch_bounds__(kBlock) void k_kinetic(long n, const double *__restrict__ P, double *__restrict__ part)
{
    double s = 0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
        s += 0.5 * P[t] * P[t];
    block_partial(s, part);
}

// per-block maximum and sum of the link force norms |F| = (sum_a F_a^2)^(1/2) over the nl
// links (p, mu, i) of the internal momenta layout; part[2 b] = max, part[2 b + 1] = sum
__global__ __launch_bounds__(256) void k_force_norm(long nl, long Vh, const double *__restrict__ F,
                                                    double *__restrict__ part)
{
    double mx = 0, sm = 0;
    for (long l = blockIdx.x * (long)blockDim.x + threadIdx.x; l < nl; l += (long)gridDim.x * blockDim.x) {
        const long pm = l / Vh, i = l - pm * Vh;
        const double *b = F + pm * 8 * Vh + i;
        double s = 0;
#pragma unroll
        for (int a = 0; a < 8; a++) s = fma(b[(long)a * Vh], b[(long)a * Vh], s);
        const double v = sqrt(s);
        mx = fmax(mx, v);
        sm += v;
    }
    __shared__ double smx[4], ssm[4];
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o, 64));
        sm += __shfl_xor(sm, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        smx[threadIdx.x >> 6] = mx;
        ssm[threadIdx.x >> 6] = sm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; w++) {
            mx = fmax(mx, smx[w]);
            sm += ssm[w];
        }
        part[2 * blockIdx.x] = mx;
        part[2 * blockIdx.x + 1] = sm;
    }
}

}  // namespace

// ---------------------------------------------------------------- host side

// maximum and mean over all links of the force norm; synchronises
int force_norms(pfmp_ctx *ctx, const double *F, double *mx, double *mean)
{
    constexpr int nb = 256;
    const long nl = 8L * ctx->g.Vh;
    double *part = (double *)ws_alloc(ctx, sizeof(double) * 2 * nb, 18);
    if (!part) return set_err(ctx, PFMP_ERR_OOM, "force norm workspace");
    hipLaunchKernelGGL(k_force_norm, dim3(nb), dim3(256), 0, ctx->stream, nl, (long)ctx->g.Vh, F, part);
    LAUNCHCHK(ctx);
    double h[2 * nb];
    HIPCHK(ctx, hipMemcpyAsync(h, part, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    double m = 0, s = 0;
    for (int b = 0; b < nb; b++) {
        m = h[2 * b] > m ? h[2 * b] : m;
        s += h[2 * b + 1];
    }
    *mx = m;
    *mean = s / (double)nl;
    return 0;
}

// F += clover force of the insertion field Phi (deferred: kept for clover_force_flush)
static int clover_force_add(pfmp_ctx *ctx, const double2 *Phi, double *F)
{
    if (ctx->clover_defer) {
        ctx->phi_pending = true;
        return 0;
    }
    const Geom &g = ctx->g;
    double *Psi = (double *)ws_alloc(ctx, sizeof(double) * 2L * 6 * kPsiReals * g.Vh, 17);
    if (!Psi) return set_err(ctx, PFMP_ERR_OOM, "force workspace");
    hipLaunchKernelGGL(k_psi_pack, dim3(nblocks(12L * g.Vh, 256)), dim3(256), 0, ctx->stream, g, Phi, Psi);
    hipLaunchKernelGGL(k_clover_force, dim3(nblocks_site(16L * g.Vh)), dim3(kBlock), 0, ctx->stream, g, ctx->U,
                       Psi, F);
    LAUNCHCHK(ctx);
    return 0;
}

void clover_force_defer(pfmp_ctx *ctx)
{
    ctx->clover_defer = true;
    ctx->phi_pending = false;
}

int clover_force_flush(pfmp_ctx *ctx, double *F)
{
    const bool pending = ctx->phi_pending;
    ctx->clover_defer = false;
    ctx->phi_pending = false;
    if (!pending) return 0;
    const double2 *Phi = (const double2 *)ws_alloc(ctx, sizeof(double2) * 2L * 6 * 9 * ctx->g.Vh, 16);
    if (!Phi) return set_err(ctx, PFMP_ERR_OOM, "force workspace");
    return clover_force_add(ctx, Phi, F);
}

// Xo = A_oo^-1 (D_eo)^dag X, Zo = A_oo^-1 D_oe Y in the spinors' precision
static int force_odd(pfmp_ctx *ctx, OpSlot &s, bool cl, const double2 *x, const double2 *y, double2 *xo, double2 *zo)
{
    int rc;
    if ((rc = clovinv64(ctx, 1, y, s.clov[1], zo, 1.0, 1.0, cl, nullptr))) return rc;
    return clovinv64(ctx, 1, x, s.clov[1], xo, -1.0, -1.0, cl, nullptr);
}
static int force_odd(pfmp_ctx *ctx, OpSlot &s, bool cl, const float2 *x, const float2 *y, float2 *xo, float2 *zo)
{
    int rc;
    if ((rc = clovinv32(ctx, 1, y, s.clovf[1], zo, 1.f, 1.f, cl, nullptr))) return rc;
    return clovinv32(ctx, 1, x, s.clovf[1], xo, -1.f, -1.f, cl, nullptr);
}

template <typename C>
static int fermion_force_t(pfmp_ctx *ctx, int op, int npairs, const void *const *X, const void *const *Y,
                           const double *coeff, int flags, double *F)
{
    if (!ctx) return PFMP_ERR_ARG;
    if (op < 0 || op >= PFMP_MAX_OPS || !ctx->ops[op].valid || !ctx->have_gauge)
        return set_err(ctx, PFMP_ERR_STATE, "fermion_force: operator not configured");
    if (int rc0 = op_ready(ctx, op)) return rc0;
    if (std::is_same<C, float2>::value)
        if (int rc0 = gauge_f32_ready(ctx)) return rc0;
    if (npairs < 0 || (npairs > 0 && (!X || !Y || !coeff)) || !F)
        return set_err(ctx, PFMP_ERR_ARG, "fermion_force: bad arguments");
    for (int q = 0; q < npairs; q++)
        if (!X[q] || !Y[q]) return set_err(ctx, PFMP_ERR_ARG, "fermion_force: null field");
    if (flags == 0) flags = PFMP_FORCE_HOP | PFMP_FORCE_CLOVER;
    const Geom &g = ctx->g;
    OpSlot &s = ctx->ops[op];
    const bool cl = s.csw != 0;
    const bool do_clov = cl && (flags & PFMP_FORCE_CLOVER);
    const bool do_hop = (flags & PFMP_FORCE_HOP) != 0;
    double2 *Phi = (double2 *)ws_alloc(ctx, sizeof(double2) * 2L * 6 * 9 * g.Vh, 16);
    if (!Phi) return set_err(ctx, PFMP_ERR_OOM, "force workspace");
    const double k2 = s.kappa * s.kappa, kc = s.kappa * s.csw;
    const double2 fe = make_double2(0, kc), fo = make_double2(0, kc * k2);   // i kappa c_sw w: w = 1 even, kappa^2 odd
    // the first insertion overwrites Phi unless earlier terms of a deferred sum are in it
    const int acc0 = ctx->clover_defer && ctx->phi_pending ? 1 : 0;
    int rc = 0;
    for (int q0 = 0; q0 < npairs; q0 += kForcePairs) {
        PairSet<C> ps{};
        ps.n = npairs - q0 < kForcePairs ? npairs - q0 : kForcePairs;
        for (int k = 0; k < ps.n; k++) {
            const C *x = (const C *)X[q0 + k], *y = (const C *)Y[q0 + k];
            // pool buffers hold an FP64 spinor, so an FP32 one fits
            C *xo = (C *)pool_get(ctx, 2300 + k), *zo = (C *)pool_get(ctx, 2300 + kForcePairs + k);
            if (!xo || !zo) return set_err(ctx, PFMP_ERR_OOM, "force workspace");
            if ((rc = force_odd(ctx, s, cl, x, y, xo, zo))) return rc;
            ps.X[k] = x;
            ps.Y[k] = y;
            ps.Xo[k] = xo;
            ps.Zo[k] = zo;
            ps.c[k] = make_double2(coeff[2 * (q0 + k)], coeff[2 * (q0 + k) + 1]);
        }
        if (do_hop)
            hipLaunchKernelGGL(k_hop_force_multi<C>, dim3(nblocks(8L * g.Vh, kBlock)), dim3(kBlock), 0, ctx->stream,
                               g, ps, ctx->U, -k2, F);
        if (do_clov)
            hipLaunchKernelGGL(k_clover_insert_multi<C>, dim3(nblocks(12L * g.Vh, kBlock)), dim3(kBlock), 0,
                               ctx->stream, g, ps, fe, fo, q0 > 0 ? 1 : acc0, Phi);
        LAUNCHCHK(ctx);
    }
    if (do_clov && npairs > 0 && (rc = clover_force_add(ctx, Phi, F))) return rc;
    return 0;
}

extern "C" int pfmp_fermion_force(pfmp_ctx *ctx, int op, int npairs, const void *const *X, const void *const *Y,
                                  const double *coeff, int flags, double *F)
{
    if (flags & PFMP_FORCE_F32)
        return fermion_force_t<float2>(ctx, op, npairs, X, Y, coeff, flags & ~PFMP_FORCE_F32, F);
    return fermion_force_t<double2>(ctx, op, npairs, X, Y, coeff, flags, F);
}

int fermion_force_f32(pfmp_ctx *ctx, int op, int npairs, const void *const *X, const void *const *Y,
                      const double *coeff, double *F)
{
    return fermion_force_t<float2>(ctx, op, npairs, X, Y, coeff, 0, F);
}

extern "C" int pfmp_logdet_force(pfmp_ctx *ctx, int op, double coef, double *F)
{
    if (!ctx) return PFMP_ERR_ARG;
    if (op < 0 || op >= PFMP_MAX_OPS || !ctx->ops[op].valid || !ctx->have_gauge)
        return set_err(ctx, PFMP_ERR_STATE, "logdet_force: operator not configured");
    if (int rc0 = op_ready(ctx, op)) return rc0;
    if (!F) return set_err(ctx, PFMP_ERR_ARG, "logdet_force: null force");
    OpSlot &s = ctx->ops[op];
    if (s.csw == 0) return 0;
    const Geom &g = ctx->g;
    double2 *Phi = (double2 *)ws_alloc(ctx, sizeof(double2) * 2L * 6 * 9 * g.Vh, 16);
    if (!Phi) return set_err(ctx, PFMP_ERR_OOM, "force workspace");
    if (!(ctx->clover_defer && ctx->phi_pending))
        HIPCHK(ctx, hipMemsetAsync(Phi, 0, sizeof(double2) * 2L * 6 * 9 * g.Vh, ctx->stream));
    double2 fac = ctimesi(make_double2(-2.0 * coef * s.kappa * s.csw, 0));
    hipLaunchKernelGGL(k_logdet_insert, dim3(nblocks(g.Vh, kBlock)), dim3(kBlock), 0, ctx->stream, g, s.clov[1], fac,
                       Phi);
    LAUNCHCHK(ctx);
    return clover_force_add(ctx, Phi, F);
}

extern "C" int pfmp_gauge_force(pfmp_ctx *ctx, double beta, double *F)
{
    if (!ctx || !F) return ctx ? set_err(ctx, PFMP_ERR_ARG, "gauge_force: null") : PFMP_ERR_ARG;
    if (!ctx->have_gauge) return set_err(ctx, PFMP_ERR_STATE, "no gauge field set");
    const Geom &g = ctx->g;
    hipLaunchKernelGGL(k_gauge_force, dim3(nblocks_site(16L * g.Vh)), dim3(kBlock), 0, ctx->stream, g, ctx->U,
                       -beta / 3.0, F);
    LAUNCHCHK(ctx);
    return 0;
}

extern "C" int pfmp_update_momenta(pfmp_ctx *ctx, double eps, const double *F, double *P)
{
    if (!ctx || !F || !P) return ctx ? set_err(ctx, PFMP_ERR_ARG, "update_momenta: null") : PFMP_ERR_ARG;
    long n = mom_reals(ctx->g);
    hipLaunchKernelGGL(k_update_momenta, dim3(nblocks(n, 256)), dim3(256), 0, ctx->stream, n, eps, F, P);
    LAUNCHCHK(ctx);
    return 0;
}

extern "C" int pfmp_update_gauge(pfmp_ctx *ctx, double eps, const double *P)
{
    if (!ctx || !P) return ctx ? set_err(ctx, PFMP_ERR_ARG, "update_gauge: null") : PFMP_ERR_ARG;
    if (!ctx->have_gauge) return set_err(ctx, PFMP_ERR_STATE, "no gauge field set");
    const Geom &g = ctx->g;
    hipLaunchKernelGGL(k_update_gauge, dim3(nblocks(2L * g.Vh * 4, kBlock)), dim3(kBlock), 0, ctx->stream, g, eps, P,
                       ctx->U);
    LAUNCHCHK(ctx);
    return rebuild_gauge_derived(ctx);
}

extern "C" int pfmp_gauge_action(pfmp_ctx *ctx, double beta, double *out)
{
    if (!ctx || !out) return ctx ? set_err(ctx, PFMP_ERR_ARG, "gauge_action: null") : PFMP_ERR_ARG;
    if (!ctx->have_gauge) return set_err(ctx, PFMP_ERR_STATE, "no gauge field set");
    const Geom &g = ctx->g;
    int nb = nblocks(2L * g.Vh, kBlock);
    double *part = (double *)ws_alloc(ctx, sizeof(double) * nb, 15);
    if (!part) return set_err(ctx, PFMP_ERR_OOM, "workspace");
    hipLaunchKernelGGL(k_plaq, dim3(nb), dim3(kBlock), 0, ctx->stream, g, ctx->U, part);
    LAUNCHCHK(ctx);
    double v;
    int rc = red_finish(ctx, part, nb, 1, &v);
    if (rc) return rc;
    *out = beta * v;
    return 0;
}

extern "C" int pfmp_kinetic(pfmp_ctx *ctx, const double *P, double *out)
{
    if (!ctx || !P || !out) return ctx ? set_err(ctx, PFMP_ERR_ARG, "kinetic: null") : PFMP_ERR_ARG;
    long n = mom_reals(ctx->g);
    int nb = 1024;
    double *part = (double *)ws_alloc(ctx, sizeof(double) * nb, 15);
    if (!part) return set_err(ctx, PFMP_ERR_OOM, "workspace");
    hipLaunchKernelGGL(k_kinetic, dim3(nb), dim3(kBlock), 0, ctx->stream, n, P, part);
    LAUNCHCHK(ctx);
    return red_finish(ctx, part, nb, 1, out);
}
