// su3.h -- 3x3 complex matrices in registers (FP64) and link access on the
// internal gauge layout.
#pragma once
#include "internal.h"

struct M3 {
    double2 e[9];
};

PFMP_HD M3 m3_zero()
{
    M3 r;
    for (int k = 0; k < 9; k++) r.e[k] = make_double2(0, 0);
    return r;
}
PFMP_HD M3 m3_eye()
{
    M3 r = m3_zero();
    r.e[0].x = r.e[4].x = r.e[8].x = 1;
    return r;
}
// a b
PFMP_HD M3 m3_mul(const M3 &a, const M3 &b)
{
    M3 r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double2 s = cmul(a.e[3 * i], b.e[j]);
            cfma(s, a.e[3 * i + 1], b.e[3 + j]);
            cfma(s, a.e[3 * i + 2], b.e[6 + j]);
            r.e[3 * i + j] = s;
        }
    return r;
}
// a b^dag
PFMP_HD M3 m3_mul_nd(const M3 &a, const M3 &b)
{
    M3 r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double2 s = cmul(a.e[3 * i], cconj(b.e[3 * j]));
            cfma(s, a.e[3 * i + 1], cconj(b.e[3 * j + 1]));
            cfma(s, a.e[3 * i + 2], cconj(b.e[3 * j + 2]));
            r.e[3 * i + j] = s;
        }
    return r;
}
// a^dag b
PFMP_HD M3 m3_mul_dn(const M3 &a, const M3 &b)
{
    M3 r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double2 s = cmulc(a.e[i], b.e[j]);
            cfmac(s, a.e[3 + i], b.e[3 + j]);
            cfmac(s, a.e[6 + i], b.e[6 + j]);
            r.e[3 * i + j] = s;
        }
    return r;
}
PFMP_HD M3 m3_dag(const M3 &a)
{
    M3 r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r.e[3 * i + j] = cconj(a.e[3 * j + i]);
    return r;
}
// a^dag when dag, else a (per-lane select, no branch)
PFMP_HD M3 m3_dag_if(const M3 &a, bool dag)
{
    M3 r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double2 d = cconj(a.e[3 * j + i]), n = a.e[3 * i + j];
            r.e[3 * i + j] = make_double2(dag ? d.x : n.x, dag ? d.y : n.y);
        }
    return r;
}
PFMP_HD M3 m3_add(const M3 &a, const M3 &b)
{
    M3 r;
    for (int k = 0; k < 9; k++) r.e[k] = cadd(a.e[k], b.e[k]);
    return r;
}
PFMP_HD M3 m3_sub(const M3 &a, const M3 &b)
{
    M3 r;
    for (int k = 0; k < 9; k++) r.e[k] = csub(a.e[k], b.e[k]);
    return r;
}
PFMP_HD M3 m3_scale(const M3 &a, double s)
{
    M3 r;
    for (int k = 0; k < 9; k++) r.e[k] = cscale(a.e[k], s);
    return r;
}
PFMP_HD M3 m3_cscale(const M3 &a, double2 s)
{
    M3 r;
    for (int k = 0; k < 9; k++) r.e[k] = cmul(a.e[k], s);
    return r;
}
PFMP_HD double2 m3_trace(const M3 &a) { return cadd(cadd(a.e[0], a.e[4]), a.e[8]); }

// Coefficients f_a = Re tr[i T_a Z] = -Im tr[T_a Z], T_a = lambda_a / 2.
PFMP_HD void lie_coeffs(const M3 &Z, double *f)
{
    const double2 *z = Z.e;
    // tr(T_a Z) = sum_ij (T_a)_ij Z_ji
    double2 t1 = cscale(cadd(z[3], z[1]), 0.5);                              // (Z10 + Z01)/2
    double2 t2 = cscale(csub(ctimesi(z[1]), ctimesi(z[3])), 0.5);            // (i Z01 - i Z10)/2
    double2 t3 = cscale(csub(z[0], z[4]), 0.5);
    double2 t4 = cscale(cadd(z[6], z[2]), 0.5);
    double2 t5 = cscale(csub(ctimesi(z[2]), ctimesi(z[6])), 0.5);
    double2 t6 = cscale(cadd(z[7], z[5]), 0.5);
    double2 t7 = cscale(csub(ctimesi(z[5]), ctimesi(z[7])), 0.5);
    double2 t8 = cscale(csub(cadd(z[0], z[4]), cscale(z[8], 2.0)), 0.5 / 1.7320508075688772935);
    f[0] = -t1.y; f[1] = -t2.y; f[2] = -t3.y; f[3] = -t4.y;
    f[4] = -t5.y; f[5] = -t6.y; f[6] = -t7.y; f[7] = -t8.y;
}

// P = sum_a p_a T_a (traceless Hermitian)
PFMP_HD M3 lie_matrix(const double *p)
{
    const double s3 = 0.57735026918962576451;   // 1/sqrt(3)
    M3 r;
    r.e[0] = make_double2(0.5 * (p[2] + p[7] * s3), 0);
    r.e[4] = make_double2(0.5 * (-p[2] + p[7] * s3), 0);
    r.e[8] = make_double2(-p[7] * s3, 0);
    r.e[1] = make_double2(0.5 * p[0], -0.5 * p[1]);
    r.e[3] = make_double2(0.5 * p[0], 0.5 * p[1]);
    r.e[2] = make_double2(0.5 * p[3], -0.5 * p[4]);
    r.e[6] = make_double2(0.5 * p[3], 0.5 * p[4]);
    r.e[5] = make_double2(0.5 * p[5], -0.5 * p[6]);
    r.e[7] = make_double2(0.5 * p[5], 0.5 * p[6]);
    return r;
}

// ------------------------------------------------------------------ coordinates

__device__ __forceinline__ void shifted(const Geom &g, const int *c, int mu, int step, int *d)
{
    d[0] = c[0]; d[1] = c[1]; d[2] = c[2]; d[3] = c[3];
    int v = d[mu] + step;
    if (v >= g.L[mu]) v -= g.L[mu];
    if (v < 0) v += g.L[mu];
    d[mu] = v;
}

__device__ __forceinline__ int parity_of(const int *c) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

// U_mu at the site with coordinates c
__device__ __forceinline__ M3 link_at(const Geom &g, const double2 *__restrict__ U, const int *c, int mu)
{
    int p = parity_of(c);
    int i = eo_index(g, c);
    M3 r;
    const double2 *b = U + ((long)(p * 4 + mu) * 9) * g.Vh + i;
    for (int k = 0; k < 9; k++) r.e[k] = b[(long)k * g.Vh];
    return r;
}

// As link_at, but when every link is in SU(3) (g.recon) only rows 1 and 2 are read and
// row 3 is their conjugate cross product (for the kernels bound by their link gathers).
__device__ __forceinline__ M3 link_at_su3(const Geom &g, const double2 *__restrict__ U, const int *c, int mu)
{
    if (!g.recon) return link_at(g, U, c, mu);
    const double2 *b = U + ((long)(parity_of(c) * 4 + mu) * 9) * g.Vh + eo_index(g, c);
    M3 r;
    for (int k = 0; k < 6; k++) r.e[k] = b[(long)k * g.Vh];
    r.e[6] = cconj(csub(cmul(r.e[1], r.e[5]), cmul(r.e[2], r.e[4])));
    r.e[7] = cconj(csub(cmul(r.e[2], r.e[3]), cmul(r.e[0], r.e[5])));
    r.e[8] = cconj(csub(cmul(r.e[0], r.e[4]), cmul(r.e[1], r.e[3])));
    return r;
}

__device__ __forceinline__ void link_store(const Geom &g, double2 *__restrict__ U, int p, int i, int mu, const M3 &m)
{
    double2 *b = U + ((long)(p * 4 + mu) * 9) * g.Vh + i;
    for (int k = 0; k < 9; k++) b[(long)k * g.Vh] = m.e[k];
}

// Plane index of (mu, nu), mu < nu: (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
PFMP_HD int plane_index(int mu, int nu) { return mu == 0 ? nu - 1 : (mu == 1 ? nu + 1 : 5); }
