/*
 * pfmp_oracle.c -- plain FP64 CPU oracle for the hot path of polynomial-filtered
 * mass-preconditioned HMC (arXiv:1609.02652).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls
 * this file; only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant with the HIP path.
 *
 * It is written to be checked by eye against the definitions, not to be fast:
 *   - full 4x4 Dirac matrices (no spin projection), neighbours recomputed from
 *     coordinates on every access;
 *   - the even-odd hopping blocks are the full-lattice hopping term restricted to
 *     one output parity;
 *   - the clover term is a dense 12x12 matrix per site, inverted by Gauss-Jordan
 *     elimination, its log-determinant taken from the LU pivots;
 *   - every force is the derivative of the operator or action by the product rule:
 *     one link at a time is moved along U -> exp(i w T_a) U and the derivative of
 *     the definition is evaluated at w = 0 (no outer-product or staple
 *     bookkeeping).
 *
 * Conventions (shared with the library only through the written interface):
 *   lattice L[4] = (Lx, Ly, Lz, Lt), all even; lexicographic site index
 *   lex = x + Lx*(y + Ly*(z + Lz*t)); parity = (x+y+z+t) mod 2;
 *   even-odd index = lex/2.  Gauge links periodic.  Fermion hops that cross the
 *   t boundary take the factor tbc (= -1 antiperiodic).
 *   Gauge field U[lex][mu][a][b], complex128.  Spinor psi[site][spin][colour].
 *   Dirac matrices: chiral basis, g_k = [[0,-i s_k],[i s_k,0]], g_4 = [[0,1],[1,0]].
 *   Lie-algebra coefficients per link: 8 reals for T_a = lambda_a / 2.
 *
 * Operator definitions follow the paper's fermion matrix M, K = M^dag M (Sec. 2.1),
 * with the Wilson hopping term (Table 3.1 "even-odd Wilson") and the clover term:
 *   D_hop psi(x) = sum_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^dag psi(x-mu)]
 *   M = A - kappa D_hop,  A = 1 + i kappa csw sum_{mu<nu} sigma_mu_nu (x) Fhat_mu_nu,
 *   Fhat = (Q - Q^dag)/8 over the four clover leaves, sigma = (i/2)[g_mu, g_nu],
 *   Mhat = A_ee - kappa^2 D_eo A_oo^-1 D_oe on even sites.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* Geometry                                                           */
/* ------------------------------------------------------------------ */

static long volume(const int *L) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void coords_of(const int *L, long lex, int *c)
{
    c[0] = (int)(lex % L[0]); lex /= L[0];
    c[1] = (int)(lex % L[1]); lex /= L[1];
    c[2] = (int)(lex % L[2]); lex /= L[2];
    c[3] = (int)lex;
}

static long lex_of(const int *L, const int *c)
{
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

static int parity_of(const int *L, long lex)
{
    int c[4];
    coords_of(L, lex, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* Site one step along +mu (step=+1) or -mu (step=-1); *fsign gets the fermion
 * boundary factor of that hop (tbc when the t coordinate wraps, else 1). */
static long neighbour(const int *L, int tbc, long lex, int mu, int step, double *fsign)
{
    int c[4];
    coords_of(L, lex, c);
    double s = 1.0;
    int v = c[mu] + step;
    if (v >= L[mu]) { v -= L[mu]; if (mu == 3) s = tbc; }
    if (v < 0) { v += L[mu]; if (mu == 3) s = tbc; }
    c[mu] = v;
    if (fsign) *fsign = s;
    return lex_of(L, c);
}

/* lex index of even-odd index i of the given parity: of the two sites 2i, 2i+1
 * (neighbours along x, Lx even) exactly one has that parity. */
static long lex_of_eo(const int *L, int parity, long i)
{
    return parity_of(L, 2 * i) == parity ? 2 * i : 2 * i + 1;
}

/* Exact index tables: lex_of_eo[p][i]; nbr[p][i][d] = even-odd index of the
 * neighbour in direction d = 2*mu (+mu) or 2*mu+1 (-mu); sign[p][i][d] = fermion
 * boundary factor of that hop. */
int or_index_maps(const int *L, int tbc, int32_t *lexeo, int32_t *nbr, int8_t *sign)
{
    long V = volume(L), Vh = V / 2;
    for (int p = 0; p < 2; p++)
        for (long i = 0; i < Vh; i++) {
            long x = lex_of_eo(L, p, i);
            lexeo[p * Vh + i] = (int32_t)x;
            for (int mu = 0; mu < 4; mu++)
                for (int b = 0; b < 2; b++) {
                    double s;
                    long y = neighbour(L, tbc, x, mu, b ? -1 : +1, &s);
                    nbr[(p * Vh + i) * 8 + 2 * mu + b] = (int32_t)(y / 2);
                    sign[(p * Vh + i) * 8 + 2 * mu + b] = (int8_t)(s < 0 ? -1 : 1);
                }
        }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Dirac algebra                                                      */
/* ------------------------------------------------------------------ */

static cplx GAM[4][4][4];          /* gamma_mu, mu = 0..3 = x,y,z,t */
static cplx G5[4][4];
static cplx SIG[4][4][4][4];       /* sigma_{mu nu} = (i/2)[g_mu, g_nu] */
static cplx LAM[8][3][3];          /* T_a = lambda_a / 2 */

static void mat4_mul(cplx a[4][4], cplx b[4][4], cplx r[4][4])
{
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx s = 0;
            for (int k = 0; k < 4; k++) s += a[i][k] * b[k][j];
            r[i][j] = s;
        }
}

__attribute__((constructor)) static void init_algebra(void)
{
    cplx pauli[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(GAM, 0, sizeof GAM);
    for (int k = 0; k < 3; k++)
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++) {
                GAM[k][i][2 + j] = -I * pauli[k][i][j];
                GAM[k][2 + i][j] = I * pauli[k][i][j];
            }
    for (int i = 0; i < 2; i++) { GAM[3][i][2 + i] = 1; GAM[3][2 + i][i] = 1; }
    cplx t1[4][4], t2[4][4];
    mat4_mul(GAM[0], GAM[1], t1);
    mat4_mul(t1, GAM[2], t2);
    mat4_mul(t2, GAM[3], G5);
    for (int m = 0; m < 4; m++)
        for (int n = 0; n < 4; n++) {
            mat4_mul(GAM[m], GAM[n], t1);
            mat4_mul(GAM[n], GAM[m], t2);
            for (int i = 0; i < 4; i++)
                for (int j = 0; j < 4; j++) SIG[m][n][i][j] = 0.5 * I * (t1[i][j] - t2[i][j]);
        }
    memset(LAM, 0, sizeof LAM);
    LAM[0][0][1] = LAM[0][1][0] = 0.5;
    LAM[1][0][1] = -0.5 * I; LAM[1][1][0] = 0.5 * I;
    LAM[2][0][0] = 0.5; LAM[2][1][1] = -0.5;
    LAM[3][0][2] = LAM[3][2][0] = 0.5;
    LAM[4][0][2] = -0.5 * I; LAM[4][2][0] = 0.5 * I;
    LAM[5][1][2] = LAM[5][2][1] = 0.5;
    LAM[6][1][2] = -0.5 * I; LAM[6][2][1] = 0.5 * I;
    LAM[7][0][0] = LAM[7][1][1] = 0.5 / sqrt(3.0); LAM[7][2][2] = -1.0 / sqrt(3.0);
}

/* Export the Dirac and Lie matrices so tests can check the algebra itself. */
void or_gamma(int mu, double *out /* 4x4 complex */)
{
    cplx (*m)[4] = mu < 4 ? GAM[mu] : G5;
    memcpy(out, m, sizeof(cplx) * 16);
}

void or_generator(int a, double *out /* 3x3 complex */) { memcpy(out, LAM[a], sizeof(cplx) * 9); }

/* ------------------------------------------------------------------ */
/* Small dense helpers                                                */
/* ------------------------------------------------------------------ */

static void m3_mul(const cplx *a, const cplx *b, cplx *r)
{
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx s = 0;
            for (int k = 0; k < 3; k++) s += a[3 * i + k] * b[3 * k + j];
            t[3 * i + j] = s;
        }
    memcpy(r, t, sizeof t);
}

static void m3_dag(const cplx *a, cplx *r)
{
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) t[3 * i + j] = conj(a[3 * j + i]);
    memcpy(r, t, sizeof t);
}

static void m3_eye(cplx *r)
{
    for (int i = 0; i < 9; i++) r[i] = (i % 4 == 0) ? 1 : 0;
}

/* t[s][a] = sum_b W[a][b] in[s][b] */
static void colour_mul(const cplx *W, const cplx *in, cplx *t)
{
    for (int s = 0; s < 4; s++)
        for (int a = 0; a < 3; a++) {
            cplx v = 0;
            for (int b = 0; b < 3; b++) v += W[3 * a + b] * in[3 * s + b];
            t[3 * s + a] = v;
        }
}

/* out[s][a] += f * sum_t (1 + pm*g)[s][t] in[t][a] */
static void spin_proj_acc(const cplx g[4][4], double pm, double f, const cplx *in, cplx *out)
{
    for (int s = 0; s < 4; s++)
        for (int a = 0; a < 3; a++) {
            cplx v = in[3 * s + a];
            for (int t = 0; t < 4; t++) v += pm * g[s][t] * in[3 * t + a];
            out[3 * s + a] += f * v;
        }
}

/* In-place Gauss-Jordan inverse of an n x n complex matrix with partial pivoting. */
static int gj_inverse(cplx *a, int n, cplx *inv)
{
    cplx w[144];
    memcpy(w, a, sizeof(cplx) * n * n);
    for (int i = 0; i < n * n; i++) inv[i] = 0;
    for (int i = 0; i < n; i++) inv[i * n + i] = 1;
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (cabs(w[r * n + c]) > cabs(w[p * n + c])) p = r;
        if (cabs(w[p * n + c]) == 0) return -1;
        if (p != c)
            for (int k = 0; k < n; k++) {
                cplx t = w[c * n + k]; w[c * n + k] = w[p * n + k]; w[p * n + k] = t;
                t = inv[c * n + k]; inv[c * n + k] = inv[p * n + k]; inv[p * n + k] = t;
            }
        cplx d = 1.0 / w[c * n + c];
        for (int k = 0; k < n; k++) { w[c * n + k] *= d; inv[c * n + k] *= d; }
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            cplx f = w[r * n + c];
            if (f == 0) continue;
            for (int k = 0; k < n; k++) { w[r * n + k] -= f * w[c * n + k]; inv[r * n + k] -= f * inv[c * n + k]; }
        }
    }
    return 0;
}

/* log det of an n x n complex matrix from LU with partial pivoting; returns the
 * complex logarithm (real part = ln|det|, imaginary part = phase). */
static cplx lu_logdet(const cplx *a, int n)
{
    cplx w[144];
    memcpy(w, a, sizeof(cplx) * n * n);
    cplx ld = 0;
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (cabs(w[r * n + c]) > cabs(w[p * n + c])) p = r;
        if (p != c) {
            for (int k = 0; k < n; k++) { cplx t = w[c * n + k]; w[c * n + k] = w[p * n + k]; w[p * n + k] = t; }
            ld += I * M_PI;
        }
        ld += clog(w[c * n + c]);
        for (int r = c + 1; r < n; r++) {
            cplx f = w[r * n + c] / w[c * n + c];
            for (int k = c; k < n; k++) w[r * n + k] -= f * w[c * n + k];
        }
    }
    return ld;
}

/* ------------------------------------------------------------------ */
/* Link access with an optional one-link derivative                   */
/* ------------------------------------------------------------------ */

/* A "link view": either the gauge field itself, or its derivative along a single
 * link (dsite, dmu), i.e. every link zero except that one, which is dU. */
typedef struct {
    const int *L;
    const cplx *U;
    long dsite;      /* -1: plain field */
    int dmu;
    const cplx *dU;
} linkview;

/* One step of a path from site s along +mu (dir = mu+1) or -mu (dir = -(mu+1)).
 * Returns the next site; sets the link's site, direction and whether it enters
 * daggered. */
static long path_step(const int *L, long s, int dir, long *lsite, int *lmu, int *dag)
{
    int mu = (dir > 0 ? dir : -dir) - 1;
    if (dir > 0) {
        *lsite = s; *lmu = mu; *dag = 0;
        return neighbour(L, 1, s, mu, +1, NULL);
    }
    long b = neighbour(L, 1, s, mu, -1, NULL);
    *lsite = b; *lmu = mu; *dag = 1;
    return b;
}

/* Ordered product of the links along a closed path of 4 steps from x.  With a
 * derivative view, the product rule: sum over the steps whose link is the
 * perturbed one, with that factor replaced by dU (or dU^dag). */
static void path_product(const linkview *lv, long x, const int *dirs, int nsteps, cplx *out)
{
    long ls[8]; int lm[8], dg[8];
    long s = x;
    for (int k = 0; k < nsteps; k++) s = path_step(lv->L, s, dirs[k], &ls[k], &lm[k], &dg[k]);
    if (lv->dsite < 0) {
        m3_eye(out);
        for (int k = 0; k < nsteps; k++) {
            cplx m[9];
            const cplx *u = lv->U + (ls[k] * 4 + lm[k]) * 9;
            if (dg[k]) m3_dag(u, m); else memcpy(m, u, sizeof m);
            m3_mul(out, m, out);
        }
        return;
    }
    for (int i = 0; i < 9; i++) out[i] = 0;
    for (int j = 0; j < nsteps; j++) {
        if (ls[j] != lv->dsite || lm[j] != lv->dmu) continue;
        cplx prod[9];
        m3_eye(prod);
        for (int k = 0; k < nsteps; k++) {
            cplx m[9];
            const cplx *u = (k == j) ? lv->dU : lv->U + (ls[k] * 4 + lm[k]) * 9;
            if (dg[k]) m3_dag(u, m); else memcpy(m, u, sizeof m);
            m3_mul(prod, m, prod);
        }
        for (int i = 0; i < 9; i++) out[i] += prod[i];
    }
}

/* The four clover leaves at x in the (mu,nu) plane, all traversed the same way
 * round: they start and end at x. */
static void leaf_dirs(int mu, int nu, int k, int *d)
{
    int m = mu + 1, n = nu + 1;
    int leaves[4][4] = {
        {+m, +n, -m, -n},
        {+n, -m, -n, +m},
        {-m, -n, +m, +n},
        {-n, +m, +n, -m},
    };
    memcpy(d, leaves[k], sizeof(int) * 4);
}

/* Fhat_{mu nu}(x) = (Q - Q^dag)/8, Q = sum of the four leaves (or its derivative). */
static void fhat(const linkview *lv, long x, int mu, int nu, cplx *F)
{
    cplx Q[9] = {0}, P[9];
    int d[4];
    for (int k = 0; k < 4; k++) {
        leaf_dirs(mu, nu, k, d);
        path_product(lv, x, d, 4, P);
        for (int i = 0; i < 9; i++) Q[i] += P[i];
    }
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) F[3 * i + j] = (Q[3 * i + j] - conj(Q[3 * j + i])) / 8.0;
}

/* Clover matrix A(x) (identity included unless deriv) as 12x12, index s*3+c. */
static void clover_site(const linkview *lv, double kappa, double csw, long x, int with_identity, cplx *A)
{
    for (int i = 0; i < 144; i++) A[i] = 0;
    if (with_identity)
        for (int i = 0; i < 12; i++) A[i * 12 + i] = 1;
    if (csw == 0) return;
    for (int mu = 0; mu < 4; mu++)
        for (int nu = mu + 1; nu < 4; nu++) {
            cplx F[9];
            fhat(lv, x, mu, nu, F);
            for (int s = 0; s < 4; s++)
                for (int t = 0; t < 4; t++) {
                    cplx sg = SIG[mu][nu][s][t];
                    if (sg == 0) continue;
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++)
                            A[(s * 3 + a) * 12 + t * 3 + b] += I * kappa * csw * sg * F[3 * a + b];
                }
        }
}

/* Wilson hopping term at one output site x, for a link view. adjoint swaps the
 * projectors (D_hop^dag).  out[12] is overwritten. */
static void hop_at(const linkview *lv, int tbc, const cplx *in, long x, int adjoint, cplx *out)
{
    const int *L = lv->L;
    for (int i = 0; i < 12; i++) out[i] = 0;
    for (int mu = 0; mu < 4; mu++) {
        double sf, sb;
        long xf = neighbour(L, tbc, x, mu, +1, &sf);
        long xb = neighbour(L, tbc, x, mu, -1, &sb);
        cplx t[12], m[9];
        const cplx *uf = NULL, *ub = NULL;
        if (lv->dsite < 0) {
            uf = lv->U + (x * 4 + mu) * 9;
            ub = lv->U + (xb * 4 + mu) * 9;
        } else {
            if (lv->dsite == x && lv->dmu == mu) uf = lv->dU;
            if (lv->dsite == xb && lv->dmu == mu) ub = lv->dU;
        }
        /* forward: (1 - g_mu) U_mu(x) psi(x+mu)   [adjoint: (1 + g_mu)] */
        if (uf) {
            colour_mul(uf, in + 12 * xf, t);
            spin_proj_acc(GAM[mu], adjoint ? +1.0 : -1.0, sf, t, out);
        }
        /* backward: (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)   [adjoint: (1 - g_mu)] */
        if (ub) {
            m3_dag(ub, m);
            colour_mul(m, in + 12 * xb, t);
            spin_proj_acc(GAM[mu], adjoint ? -1.0 : +1.0, sb, t, out);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Operator context                                                   */
/* ------------------------------------------------------------------ */

typedef struct {
    int L[4];
    int tbc;
    long V, Vh;
    const cplx *U;      /* borrowed, [V][4][3][3] */
    double kappa, csw;
    cplx *A;            /* [V][144] */
    cplx *Ainv;         /* [V][144] */
    cplx *logdet;       /* [V] complex log det A(x) */
    void *occ;          /* leaf occurrences per link, built on first force call */
} or_op;

void *or_op_create(const int *L, int tbc, const double *U, double kappa, double csw)
{
    for (int m = 0; m < 4; m++)
        if (L[m] < 4 || (L[m] & 1)) return NULL;
    or_op *op = calloc(1, sizeof *op);
    memcpy(op->L, L, sizeof op->L);
    op->tbc = tbc;
    op->V = volume(L);
    op->Vh = op->V / 2;
    op->U = (const cplx *)U;
    op->kappa = kappa;
    op->csw = csw;
    op->A = malloc(sizeof(cplx) * 144 * op->V);
    op->Ainv = malloc(sizeof(cplx) * 144 * op->V);
    op->logdet = malloc(sizeof(cplx) * op->V);
    linkview lv = {op->L, op->U, -1, 0, NULL};
#pragma omp parallel for schedule(static)
    for (long x = 0; x < op->V; x++) {
        clover_site(&lv, kappa, csw, x, 1, op->A + 144 * x);
        gj_inverse(op->A + 144 * x, 12, op->Ainv + 144 * x);
        op->logdet[x] = lu_logdet(op->A + 144 * x, 12);
    }
    return op;
}

void or_op_free(void *p)
{
    or_op *op = p;
    if (!op) return;
    free(op->A); free(op->Ainv); free(op->logdet); free(op->occ); free(op);
}

/* Dense clover matrix, its inverse and complex log det at one site. */
void or_clover_at(void *p, long lex, double *A, double *Ainv, double *logdet)
{
    or_op *op = p;
    if (A) memcpy(A, op->A + 144 * lex, sizeof(cplx) * 144);
    if (Ainv) memcpy(Ainv, op->Ainv + 144 * lex, sizeof(cplx) * 144);
    if (logdet) memcpy(logdet, op->logdet + lex, sizeof(cplx));
}

/* Full-lattice hopping term (or its adjoint), restricted to output parity
 * out_parity (-1: every site). */
static void hop_full(const or_op *op, const cplx *in, cplx *out, int adjoint, int out_parity)
{
    linkview lv = {op->L, op->U, -1, 0, NULL};
#pragma omp parallel for schedule(static)
    for (long x = 0; x < op->V; x++) {
        if (out_parity >= 0 && parity_of(op->L, x) != out_parity) {
            for (int i = 0; i < 12; i++) out[12 * x + i] = 0;
            continue;
        }
        hop_at(&lv, op->tbc, in, x, adjoint, out + 12 * x);
    }
}

void or_hop_full(void *p, int adjoint, const double *in, double *out)
{
    hop_full(p, (const cplx *)in, (cplx *)out, adjoint, -1);
}

static void embed(const or_op *op, int parity, const cplx *eo, cplx *full)
{
    memset(full, 0, sizeof(cplx) * 12 * op->V);
    for (long i = 0; i < op->Vh; i++)
        memcpy(full + 12 * lex_of_eo(op->L, parity, i), eo + 12 * i, sizeof(cplx) * 12);
}

static void extract(const or_op *op, int parity, const cplx *full, cplx *eo)
{
    for (long i = 0; i < op->Vh; i++)
        memcpy(eo + 12 * i, full + 12 * lex_of_eo(op->L, parity, i), sizeof(cplx) * 12);
}

/* Even-odd hopping block: output parity out_parity from an input field on the
 * other parity (D_eo for out_parity = 0, D_oe for 1; adjoint: the blocks of
 * D_hop^dag). */
void or_hop_eo(void *p, int out_parity, int adjoint, const double *in, double *out)
{
    or_op *op = p;
    cplx *fi = malloc(sizeof(cplx) * 12 * op->V), *fo = malloc(sizeof(cplx) * 12 * op->V);
    embed(op, 1 - out_parity, (const cplx *)in, fi);
    hop_full(op, fi, fo, adjoint, out_parity);
    extract(op, out_parity, fo, (cplx *)out);
    free(fi); free(fo);
}

/* Site-local clover (or its inverse) on one parity. */
void or_apply_clover(void *p, int parity, int inverse, const double *in_, double *out_)
{
    or_op *op = p;
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    for (long i = 0; i < op->Vh; i++) {
        const cplx *m = (inverse ? op->Ainv : op->A) + 144 * lex_of_eo(op->L, parity, i);
        cplx t[12];
        for (int r = 0; r < 12; r++) {
            cplx s = 0;
            for (int c = 0; c < 12; c++) s += m[r * 12 + c] * in[12 * i + c];
            t[r] = s;
        }
        memcpy(out + 12 * i, t, sizeof t);
    }
}

/* Mhat = A_ee - kappa^2 D_eo A_oo^-1 D_oe; dagger: A_ee - kappa^2 (D_oe)^dag A_oo^-1 (D_eo)^dag. */
void or_apply_M(void *p, int dagger, const double *in, double *out)
{
    or_op *op = p;
    long n = 12 * op->Vh;
    cplx *to = malloc(sizeof(cplx) * n), *te = malloc(sizeof(cplx) * n), *ae = malloc(sizeof(cplx) * n);
    or_hop_eo(op, 1, dagger, in, (double *)to);
    or_apply_clover(op, 1, 1, (double *)to, (double *)to);
    or_hop_eo(op, 0, dagger, (double *)to, (double *)te);
    or_apply_clover(op, 0, 0, in, (double *)ae);
    double k2 = op->kappa * op->kappa;
    for (long i = 0; i < n; i++) ((cplx *)out)[i] = ae[i] - k2 * te[i];
    free(to); free(te); free(ae);
}

/* The hop D_oe psi (mode 0: output on odd sites) or Mhat psi (mode 1: output on even
 * sites; dagger selects Mhat^dag) evaluated at n chosen output sites only, straight
 * from the definitions and without an operator context: for an even site x the
 * clover matrix A(x) and, for each of its eight odd neighbours y, A(y) and its
 * inverse are built on the spot, and (D_oe psi)(y) is the hopping term at y.  This
 * gives the oracle's value at sampled sites of lattices too large for the dense
 * per-site clover storage of the operator context.  in: even-parity field
 * [Vh][12] complex; sites: even-odd indices of the output parity; out: [n][12]. */
int or_sample_sites(const int *L, int tbc, const double *U, double kappa, double csw, int mode, int dagger,
                    const double *in_, long n, const long *sites, double *out_)
{
    for (int m = 0; m < 4; m++)
        if (L[m] < 4 || (L[m] & 1)) return -1;
    const long V = volume(L), Vh = V / 2;
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    linkview lv = {L, (const cplx *)U, -1, 0, NULL};
    cplx *fi = calloc(12 * V, sizeof(cplx)), *fs = calloc(12 * V, sizeof(cplx));
    if (!fi || !fs) { free(fi); free(fs); return -2; }
    for (long i = 0; i < Vh; i++) memcpy(fi + 12 * lex_of_eo(L, 0, i), in + 12 * i, sizeof(cplx) * 12);
    for (long k = 0; k < n; k++) {
        if (sites[k] < 0 || sites[k] >= Vh) { free(fi); free(fs); return -1; }
        if (mode == 0) {
            hop_at(&lv, tbc, fi, lex_of_eo(L, 1, sites[k]), dagger, out + 12 * k);
            continue;
        }
        const long x = lex_of_eo(L, 0, sites[k]);
        long nb[8];
        for (int mu = 0; mu < 4; mu++)
            for (int st = 0; st < 2; st++) {
                double sg;
                long y = neighbour(L, tbc, x, mu, st ? -1 : +1, &sg);
                nb[2 * mu + st] = y;
                cplx t[12], A[144], Ai[144];
                hop_at(&lv, tbc, fi, y, dagger, t);
                clover_site(&lv, kappa, csw, y, 1, A);
                if (gj_inverse(A, 12, Ai)) { free(fi); free(fs); return -3; }
                for (int r = 0; r < 12; r++) {
                    cplx acc = 0;
                    for (int c = 0; c < 12; c++) acc += Ai[r * 12 + c] * t[c];
                    fs[12 * y + r] = acc;
                }
            }
        cplx te[12], A[144];
        hop_at(&lv, tbc, fs, x, dagger, te);
        clover_site(&lv, kappa, csw, x, 1, A);
        for (int r = 0; r < 12; r++) {
            cplx ae = 0;
            for (int c = 0; c < 12; c++) ae += A[r * 12 + c] * fi[12 * x + c];
            out[12 * k + r] = ae - kappa * kappa * te[r];
        }
        for (int j = 0; j < 8; j++) memset(fs + 12 * nb[j], 0, sizeof(cplx) * 12);
    }
    free(fi);
    free(fs);
    return 0;
}

/* K = Mhat^dag Mhat */
void or_apply_K(void *p, const double *in, double *out)
{
    or_op *op = p;
    cplx *t = malloc(sizeof(cplx) * 12 * op->Vh);
    or_apply_M(op, 0, in, (double *)t);
    or_apply_M(op, 1, (double *)t, out);
    free(t);
}

/* ------------------------------------------------------------------ */
/* Vector helpers                                                     */
/* ------------------------------------------------------------------ */

static cplx vdot(const cplx *a, const cplx *b, long n)
{
    cplx s = 0;
    for (long i = 0; i < n; i++) s += conj(a[i]) * b[i];
    return s;
}

static double norm2(const cplx *a, long n)
{
    double s = 0;
    for (long i = 0; i < n; i++) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

/* ------------------------------------------------------------------ */
/* Solvers (paper Sec. 2.1: CG on K; App. C: shifted inverses)        */
/* ------------------------------------------------------------------ */

/* Textbook conjugate gradient for K x = b, zero initial guess; stops when the
 * recursive residual satisfies |r| <= tol |b|, then reports the true residual. */
int or_cg(void *p, const double *b_, double *x_, double tol, int maxiter, int *iters, double *true_res)
{
    or_op *op = p;
    long n = 12 * op->Vh;
    const cplx *b = (const cplx *)b_;
    cplx *x = (cplx *)x_;
    cplx *r = malloc(sizeof(cplx) * n), *pv = malloc(sizeof(cplx) * n), *Ap = malloc(sizeof(cplx) * n);
    for (long i = 0; i < n; i++) { x[i] = 0; r[i] = b[i]; pv[i] = b[i]; }
    double bb = norm2(b, n), rr = bb;
    int k = 0, rc = 0;
    while (rr > tol * tol * bb) {
        if (k >= maxiter) { rc = -3; break; }
        or_apply_K(op, (double *)pv, (double *)Ap);
        double pAp = creal(vdot(pv, Ap, n));
        double alpha = rr / pAp;
        for (long i = 0; i < n; i++) { x[i] += alpha * pv[i]; r[i] -= alpha * Ap[i]; }
        double rr1 = norm2(r, n);
        double beta = rr1 / rr;
        rr = rr1;
        for (long i = 0; i < n; i++) pv[i] = r[i] + beta * pv[i];
        k++;
    }
    or_apply_K(op, x_, (double *)Ap);
    for (long i = 0; i < n; i++) r[i] = b[i] - Ap[i];
    if (iters) *iters = k;
    if (true_res) *true_res = sqrt(norm2(r, n) / bb);
    free(r); free(pv); free(Ap);
    return rc;
}

/* (K - z) v */
static void apply_K_shift(or_op *op, cplx z, const cplx *in, cplx *out)
{
    or_apply_K(op, (const double *)in, (double *)out);
    for (long i = 0; i < 12 * op->Vh; i++) out[i] -= z * in[i];
}

/* Solve (K - z) x = b for one complex shift z by CG on the normal equations
 * (CGNR): (K - z)^dag = K - conj(z).  Stops on the true residual |b-(K-z)x| <= tol|b|. */
int or_cg_shift(void *p, double zre, double zim, const double *b_, double *x_, double tol, int maxiter,
                int *iters, double *true_res)
{
    or_op *op = p;
    long n = 12 * op->Vh;
    cplx z = zre + I * zim;
    const cplx *b = (const cplx *)b_;
    cplx *x = (cplx *)x_;
    cplx *s = calloc(n, sizeof(cplx)), *r = calloc(n, sizeof(cplx)), *pv = calloc(n, sizeof(cplx)),
         *q = calloc(n, sizeof(cplx));
    for (long i = 0; i < n; i++) { x[i] = 0; s[i] = b[i]; }
    apply_K_shift(op, conj(z), s, r);
    memcpy(pv, r, sizeof(cplx) * n);
    double bb = norm2(b, n), rr = norm2(r, n), ss = bb;
    int k = 0, rc = 0;
    while (ss > tol * tol * bb) {
        if (k >= maxiter) { rc = -3; break; }
        apply_K_shift(op, z, pv, q);
        double alpha = rr / norm2(q, n);
        for (long i = 0; i < n; i++) { x[i] += alpha * pv[i]; s[i] -= alpha * q[i]; }
        ss = norm2(s, n);
        apply_K_shift(op, conj(z), s, r);
        double rr1 = norm2(r, n);
        double beta = rr1 / rr;
        rr = rr1;
        for (long i = 0; i < n; i++) pv[i] = r[i] + beta * pv[i];
        k++;
    }
    apply_K_shift(op, z, x, q);
    for (long i = 0; i < n; i++) s[i] = b[i] - q[i];
    if (iters) *iters = k;
    if (true_res) *true_res = sqrt(norm2(s, n) / bb);
    free(s); free(r); free(pv); free(q);
    return rc;
}

/* Product-form polynomial (App. A): out = norm * prod_k (K - z_k) in, factors
 * applied in the order given (k = 0 first).  roots: 2n doubles (re, im). */
void or_apply_poly(void *p, int n, const double *roots, double nre, double nim, const double *in, double *out)
{
    or_op *op = p;
    long len = 12 * op->Vh;
    cplx *a = malloc(sizeof(cplx) * len), *b = malloc(sizeof(cplx) * len);
    memcpy(a, in, sizeof(cplx) * len);
    for (int k = 0; k < n; k++) {
        apply_K_shift(op, roots[2 * k] + I * roots[2 * k + 1], a, b);
        cplx *t = a; a = b; b = t;
    }
    cplx nm = nre + I * nim;
    for (long i = 0; i < len; i++) ((cplx *)out)[i] = nm * a[i];
    free(a); free(b);
}

/* CG on the Hermitian positive product operator B = norm * prod_k (K - z_k)
 * (roots closed under conjugation, the product then being K times a real
 * polynomial positive on the spectrum).  Used for [K P(K)]^-1 directly. */
int or_cg_poly(void *p, int n, const double *roots, double nre, double nim, const double *b_, double *x_,
               double tol, int maxiter, int *iters, double *true_res)
{
    or_op *op = p;
    long len = 12 * op->Vh;
    const cplx *b = (const cplx *)b_;
    cplx *x = (cplx *)x_;
    cplx *r = malloc(sizeof(cplx) * len), *pv = malloc(sizeof(cplx) * len), *Ap = malloc(sizeof(cplx) * len);
    for (long i = 0; i < len; i++) { x[i] = 0; r[i] = b[i]; pv[i] = b[i]; }
    double bb = norm2(b, len), rr = bb;
    int k = 0, rc = 0;
    while (rr > tol * tol * bb) {
        if (k >= maxiter) { rc = -3; break; }
        or_apply_poly(op, n, roots, nre, nim, (double *)pv, (double *)Ap);
        double pAp = creal(vdot(pv, Ap, len));
        double alpha = rr / pAp;
        for (long i = 0; i < len; i++) { x[i] += alpha * pv[i]; r[i] -= alpha * Ap[i]; }
        double rr1 = norm2(r, len);
        double beta = rr1 / rr;
        rr = rr1;
        for (long i = 0; i < len; i++) pv[i] = r[i] + beta * pv[i];
        k++;
    }
    or_apply_poly(op, n, roots, nre, nim, x_, (double *)Ap);
    for (long i = 0; i < len; i++) r[i] = b[i] - Ap[i];
    if (iters) *iters = k;
    if (true_res) *true_res = sqrt(norm2(r, len) / bb);
    free(r); free(pv); free(Ap);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Actions                                                            */
/* ------------------------------------------------------------------ */

/* Wilson gauge action S_G = beta * sum_{x, mu<nu} (1 - Re tr U_P / 3). */
double or_gauge_action(const int *L, const double *U, double beta)
{
    linkview lv = {L, (const cplx *)U, -1, 0, NULL};
    long V = volume(L);
    double s = 0;
#pragma omp parallel for reduction(+ : s)
    for (long x = 0; x < V; x++)
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                int d[4];
                leaf_dirs(mu, nu, 0, d);
                cplx P[9];
                path_product(&lv, x, d, 4, P);
                s += 1.0 - creal(P[0] + P[4] + P[8]) / 3.0;
            }
    return beta * s;
}

/* Average plaquette Re tr U_P / 3 */
double or_plaquette(const int *L, const double *U)
{
    long V = volume(L);
    return 1.0 - or_gauge_action(L, U, 1.0) / (6.0 * V);
}

/* S_det = -2 sum_{x odd} ln det A(x) (two flavours; det M = det A_oo det Mhat). */
double or_logdet_action(void *p)
{
    or_op *op = p;
    double s = 0;
    for (long i = 0; i < op->Vh; i++) s += creal(op->logdet[lex_of_eo(op->L, 1, i)]);
    return -2.0 * s;
}

/* ------------------------------------------------------------------ */
/* Forces by the product rule                                         */
/* ------------------------------------------------------------------ */

/* dU = i T_a U for the generator a */
static void lie_deriv(const cplx *U, int a, cplx *dU)
{
    cplx t[9];
    for (int i = 0; i < 9; i++) t[i] = I * LAM[a][i / 3][i % 3];
    m3_mul(t, U, dU);
}

/* Where each link occurs in the clover leaves: for every site x, plane (mu<nu)
 * and leaf k, the four links of the leaf are found by walking it, and (x, plane,
 * leaf) is recorded under each of them.  Every link ends up in exactly 24 leaves
 * (3 planes x 2 plaquettes x 4 corners). */
typedef struct { long x; int mu, nu, leaf; } occ_t;
#define OCC_PER_LINK 24

static occ_t *build_occurrences(const int *L)
{
    long V = volume(L);
    occ_t *occ = malloc(sizeof(occ_t) * OCC_PER_LINK * 4 * V);
    int *cnt = calloc(4 * V, sizeof(int));
    for (long x = 0; x < V; x++)
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++)
                for (int k = 0; k < 4; k++) {
                    int d[4];
                    leaf_dirs(mu, nu, k, d);
                    long s = x;
                    for (int j = 0; j < 4; j++) {
                        long ls; int lm, dg;
                        s = path_step(L, s, d[j], &ls, &lm, &dg);
                        long link = ls * 4 + lm;
                        if (cnt[link] >= OCC_PER_LINK) { free(occ); free(cnt); return NULL; }
                        occ_t o = {x, mu, nu, k};
                        occ[link * OCC_PER_LINK + cnt[link]++] = o;
                    }
                }
    free(cnt);
    return occ;
}

/* Derivative of the clover matrices along one link: the distinct sites x whose
 * A(x) depends on the link, and dA(x) = i kappa csw sum sigma (x) dFhat there,
 * dFhat = (dQ - dQ^dag)/8, dQ by the product rule over the leaves holding the link. */
#define MAXS OCC_PER_LINK
static int clover_deriv(const linkview *dv, const occ_t *occ, double kappa, double csw, long *sites, cplx *dA)
{
    int ns = 0;
    cplx dQ[MAXS][6][9];
    memset(dQ, 0, sizeof dQ);
    for (int o = 0; o < OCC_PER_LINK; o++) {
        const occ_t *oc = occ + o;
        int si = -1;
        for (int t = 0; t < ns; t++)
            if (sites[t] == oc->x) si = t;
        if (si < 0) { si = ns; sites[ns++] = oc->x; }
        int d[4];
        leaf_dirs(oc->mu, oc->nu, oc->leaf, d);
        cplx P[9];
        path_product(dv, oc->x, d, 4, P);
        int pl = oc->mu == 0 ? oc->nu - 1 : (oc->mu == 1 ? oc->nu + 1 : 5);
        for (int i = 0; i < 9; i++) dQ[si][pl][i] += P[i];
    }
    for (int t = 0; t < ns; t++) {
        cplx *A = dA + 144 * t;
        for (int i = 0; i < 144; i++) A[i] = 0;
        int pl = 0;
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++, pl++) {
                cplx F[9];
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++)
                        F[3 * i + j] = (dQ[t][pl][3 * i + j] - conj(dQ[t][pl][3 * j + i])) / 8.0;
                for (int s = 0; s < 4; s++)
                    for (int r = 0; r < 4; r++) {
                        cplx sg = SIG[mu][nu][s][r];
                        if (sg == 0) continue;
                        for (int a = 0; a < 3; a++)
                            for (int b = 0; b < 3; b++)
                                A[(s * 3 + a) * 12 + r * 3 + b] += I * kappa * csw * sg * F[3 * a + b];
                    }
            }
    }
    return ns;
}

static occ_t *op_occurrences(or_op *op);

/*
 * F[(x*4+mu)*8 + a] += sum_p Re[ c_p X_p^dag (d Mhat / d w) Y_p ],
 * with U_mu(x) -> exp(i w T_a) U_mu(x).
 *
 * Mhat = A_ee - kappa^2 D_eo A_oo^-1 D_oe, so by the product rule
 *   X^dag dMhat Y = X^dag dA_ee Y - kappa^2 X^dag dD_eo Z + kappa^2 Xo^dag dA_oo Z
 *                   - kappa^2 Xo^dag dD_oe Y,
 * with Z = A_oo^-1 D_oe Y and Xo = A_oo^-1 (D_eo)^dag X (A is Hermitian).  On the
 * full lattice, with Lf = (X | Xo) and Rf = (Y | Z) on (even | odd) sites, this is
 *   sum_x Lf(x)^dag [ w(x) dA(x) Rf(x) - kappa^2 (dD_hop Rf)(x) ],  w = 1 (even), kappa^2 (odd).
 * Each derivative is evaluated on the definition with a one-link view.
 * links: optional list of link indices x*4+mu to evaluate (nlinks <= 0: all).
 */
void or_force_bilinear(void *p, int npairs, const double *const *Xs, const double *const *Ys, const double *coef,
                       double *F, long nlinks, const int64_t *links)
{
    or_op *op = p;
    long V = op->V, Vh = op->Vh;
    double k2 = op->kappa * op->kappa;
    occ_t *occ = op_occurrences(op);
    cplx *Lf = calloc(12 * V * npairs, sizeof(cplx)), *Rf = calloc(12 * V * npairs, sizeof(cplx));
    cplx *tmp = malloc(sizeof(cplx) * 12 * Vh);
    for (int q = 0; q < npairs; q++) {
        cplx *Lq = Lf + 12 * V * q, *Rq = Rf + 12 * V * q;
        const cplx *X = (const cplx *)Xs[q], *Y = (const cplx *)Ys[q];
        for (long i = 0; i < Vh; i++) {
            memcpy(Lq + 12 * lex_of_eo(op->L, 0, i), X + 12 * i, sizeof(cplx) * 12);
            memcpy(Rq + 12 * lex_of_eo(op->L, 0, i), Y + 12 * i, sizeof(cplx) * 12);
        }
        or_hop_eo(op, 1, 0, Ys[q], (double *)tmp);
        or_apply_clover(op, 1, 1, (double *)tmp, (double *)tmp);
        for (long i = 0; i < Vh; i++) memcpy(Rq + 12 * lex_of_eo(op->L, 1, i), tmp + 12 * i, sizeof(cplx) * 12);
        or_hop_eo(op, 1, 1, Xs[q], (double *)tmp);
        or_apply_clover(op, 1, 1, (double *)tmp, (double *)tmp);
        for (long i = 0; i < Vh; i++) memcpy(Lq + 12 * lex_of_eo(op->L, 1, i), tmp + 12 * i, sizeof(cplx) * 12);
    }
    free(tmp);

    long nl = nlinks > 0 ? nlinks : 4 * V;
#pragma omp parallel for schedule(dynamic, 4)
    for (long li = 0; li < nl; li++) {
        long link = nlinks > 0 ? links[li] : li;
        long y = link / 4;
        int mu = (int)(link % 4);
        long hs[2] = {y, neighbour(op->L, 1, y, mu, +1, NULL)};
        long sites[MAXS];
        cplx *dA = malloc(sizeof(cplx) * 144 * MAXS);
        for (int a = 0; a < 8; a++) {
            cplx dU[9];
            lie_deriv(op->U + (y * 4 + mu) * 9, a, dU);
            linkview dv = {op->L, op->U, y, mu, dU};
            int ns = op->csw != 0 ? clover_deriv(&dv, occ + link * OCC_PER_LINK, op->kappa, op->csw, sites, dA) : 0;
            double total = 0;
            for (int q = 0; q < npairs; q++) {
                const cplx *Lq = Lf + 12 * V * q, *Rq = Rf + 12 * V * q;
                cplx val = 0;
                for (int t = 0; t < ns; t++) {
                    long x = sites[t];
                    double w = parity_of(op->L, x) == 0 ? 1.0 : k2;
                    cplx v[12];
                    for (int r = 0; r < 12; r++) {
                        cplx s = 0;
                        for (int c = 0; c < 12; c++) s += dA[144 * t + r * 12 + c] * Rq[12 * x + c];
                        v[r] = w * s;
                    }
                    val += vdot(Lq + 12 * x, v, 12);
                }
                for (int h = 0; h < 2; h++) {
                    cplx v[12];
                    hop_at(&dv, op->tbc, Rq, hs[h], 0, v);
                    val -= k2 * vdot(Lq + 12 * hs[h], v, 12);
                }
                total += creal((coef[2 * q] + I * coef[2 * q + 1]) * val);
            }
            F[link * 8 + a] += total;
        }
        free(dA);
    }
    free(Lf); free(Rf);
}

/* F += coef * d/dw of S_det = -2 sum_{x odd} ln det A(x):  -2 sum tr[A^-1 dA]. */
void or_force_logdet(void *p, double coef, double *F, long nlinks, const int64_t *links)
{
    or_op *op = p;
    if (op->csw == 0) return;
    occ_t *occ = op_occurrences(op);
    long nl = nlinks > 0 ? nlinks : 4 * op->V;
#pragma omp parallel for schedule(dynamic, 4)
    for (long li = 0; li < nl; li++) {
        long link = nlinks > 0 ? links[li] : li;
        long y = link / 4;
        int mu = (int)(link % 4);
        long sites[MAXS];
        cplx *dA = malloc(sizeof(cplx) * 144 * MAXS);
        for (int a = 0; a < 8; a++) {
            cplx dU[9];
            lie_deriv(op->U + (y * 4 + mu) * 9, a, dU);
            linkview dv = {op->L, op->U, y, mu, dU};
            int ns = clover_deriv(&dv, occ + link * OCC_PER_LINK, op->kappa, op->csw, sites, dA);
            cplx val = 0;
            for (int t = 0; t < ns; t++) {
                if (parity_of(op->L, sites[t]) != 1) continue;
                const cplx *Ai = op->Ainv + 144 * sites[t];
                for (int r = 0; r < 12; r++)
                    for (int c = 0; c < 12; c++) val += Ai[r * 12 + c] * dA[144 * t + c * 12 + r];
            }
            F[link * 8 + a] += coef * (-2.0) * creal(val);
        }
        free(dA);
    }
}

/* F += d/dw of the Wilson gauge action: -(beta/3) sum over the plaquettes holding
 * the link of Re tr dU_P (plaquette = leaf 0 of a plane mu<nu at its corner x). */
void or_force_gauge(const int *L, const double *U_, double beta, double *F, long nlinks, const int64_t *links)
{
    const cplx *U = (const cplx *)U_;
    long V = volume(L);
    occ_t *occ = build_occurrences(L);
    long nl = nlinks > 0 ? nlinks : 4 * V;
#pragma omp parallel for schedule(dynamic, 16)
    for (long li = 0; li < nl; li++) {
        long link = nlinks > 0 ? links[li] : li;
        long y = link / 4;
        int mu = (int)(link % 4);
        for (int a = 0; a < 8; a++) {
            cplx dU[9];
            lie_deriv(U + (y * 4 + mu) * 9, a, dU);
            linkview dv = {L, U, y, mu, dU};
            double val = 0;
            for (int o = 0; o < OCC_PER_LINK; o++) {
                const occ_t *oc = occ + link * OCC_PER_LINK + o;
                if (oc->leaf != 0) continue;
                int d[4];
                leaf_dirs(oc->mu, oc->nu, 0, d);
                cplx P[9];
                path_product(&dv, oc->x, d, 4, P);
                val += creal(P[0] + P[4] + P[8]);
            }
            F[link * 8 + a] += -beta / 3.0 * val;
        }
    }
    free(occ);
}

/* ------------------------------------------------------------------ */
/* Integrator updates (paper App. B, atomic steps T and S)            */
/* ------------------------------------------------------------------ */

/* exp(Q) of a 3x3 complex matrix by its Taylor series, summed until the terms
 * stop changing the result (arguments here have norm well below 10). */
static void expm3(const cplx *Q, cplx *E)
{
    cplx term[9], t2[9];
    m3_eye(E);
    m3_eye(term);
    for (int k = 1; k < 60; k++) {
        m3_mul(term, Q, t2);
        double mx = 0;
        for (int i = 0; i < 9; i++) {
            term[i] = t2[i] / k;
            E[i] += term[i];
            if (cabs(term[i]) > mx) mx = cabs(term[i]);
        }
        if (mx < 1e-300 || (k > 4 && mx < 1e-18)) break;
    }
}

/* T[eps]: U_mu(x) <- exp(i eps P_mu(x)) U_mu(x), P = sum_a p_a T_a. */
void or_update_gauge(const int *L, double eps, const double *P, double *U_)
{
    cplx *U = (cplx *)U_;
    long n = 4 * volume(L);
#pragma omp parallel for schedule(static)
    for (long l = 0; l < n; l++) {
        cplx Q[9] = {0}, E[9];
        for (int a = 0; a < 8; a++)
            for (int i = 0; i < 9; i++) Q[i] += I * eps * P[l * 8 + a] * LAM[a][i / 3][i % 3];
        expm3(Q, E);
        m3_mul(E, U + 9 * l, U + 9 * l);
    }
}

/* S[eps]: P <- P - eps F (coefficients). */
void or_update_momenta(long nlinks, double eps, const double *F, double *P)
{
    for (long i = 0; i < 8 * nlinks; i++) P[i] -= eps * F[i];
}

/* Kinetic term sum tr P^2 = (1/2) sum_a p_a^2 (tr T_a T_b = delta_ab / 2). */
double or_kinetic(long nlinks, const double *P)
{
    cplx Pm[9], P2[9];
    double s = 0;
    for (long l = 0; l < nlinks; l++) {
        for (int i = 0; i < 9; i++) {
            Pm[i] = 0;
            for (int a = 0; a < 8; a++) Pm[i] += P[l * 8 + a] * LAM[a][i / 3][i % 3];
        }
        m3_mul(Pm, Pm, P2);
        s += creal(P2[0] + P2[4] + P2[8]);
    }
    return s;
}

static occ_t *op_occurrences(or_op *op)
{
    if (!op->occ) op->occ = build_occurrences(op->L);
    return op->occ;
}
