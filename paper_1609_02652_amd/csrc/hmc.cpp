// hmc.cpp -- PF-MP HMC driver (paper Sec. 2.1 HMC, eq. pfmp_action, App. B
// generalized multi-scale integrator, App. C forces), composed from the C-ABI
// kernels.  Host code only: every lattice operation is a libpfmp launch.
//
// Action: S = S_G + S_det + sum_j S_j, with S_det = -2 sum_{x odd} ln det A(x)
// of the target operator (det M = det A_oo det Mhat) and the filter terms
//   POLY      phi^dag P(J) phi,         P = a_n prod_k (J - z_k)
//   POLYCORR  phi^dag [J P(J)]^-1 phi = (1/a_n) sum_{i=1}^{n+1} r_i phi^dag (J - z_i)^-1 phi, z_{n+1} = 0
//   RATIO     phi^dag W^dag K_b^-1 W phi
//   HEAVY     phi^dag J^-1 phi
// Forces (coefficients f_a = dS/dw along U -> exp(i w T_a) U), built from the
// bilinear primitive Re[c X^dag dMhat Y] with Re[c X^dag dJ Y] =
// Re[c (W X)^dag dW Y] + Re[conj(c) (W Y)^dag dW X]:
//   POLY      sum_i Re[eta_i^dag dJ chi_i], chi_i = a_n prod_{j>i}(J - z_j) phi, eta_i = prod_{j<i}(J - z_j^*) phi
//   POLYCORR  -(1/a_n) sum_i r_i x_{i*}^dag dJ x_i, x_i = (J - z_i)^-1 phi, z_{i*} = conj(z_i)
//   RATIO     2 Re[X^dag dW phi] - 2 Re[(M_b X)^dag dM_b X], X = K_b^-1 W phi
//   HEAVY     -2 Re[(W X)^dag dW X], X = J^-1 phi
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <numeric>
#include <vector>

#include "internal.h"

using cd = std::complex<double>;

namespace {

constexpr double kOmelyanLambda = 0.1931833275037836;

struct Scheme {
    std::vector<int64_t> T;
    std::vector<double> S;
};

// n-step 2MN S[lh] T[h/2] S[(1-2l)h] T[h/2] S[lh] with adjacent space steps merged;
// time steps in ticks of tau / L (L a multiple of 2n).
Scheme omelyan(int n, int64_t L, double tau, double lam)
{
    Scheme s;
    double h = tau / n;
    int64_t half = L / (2 * n);
    s.T.push_back(0);
    s.S.push_back(lam * h);
    for (int k = 0; k < n; k++) {
        s.T.push_back(half);
        s.S.push_back((1 - 2 * lam) * h);
        s.T.push_back(half);
        s.S.push_back((k < n - 1 ? 2 * lam : lam) * h);
    }
    return s;
}

int64_t lcm64(int64_t a, int64_t b) { return a / std::gcd(a, b) * b; }

struct Ctx {
    pfmp_ctx *c;
    const pfmp_hmc_spec *sp;
    long long mhalf = 0;       // Mhat applications (2 per Khat)
    long long iters = 0;
};

int chk_spec(pfmp_ctx *ctx, const pfmp_hmc_spec *sp)
{
    if (!sp || sp->nterms < 0 || sp->nterms > PFMP_MAX_TERMS || (sp->nterms > 0 && !sp->terms))
        return set_err(ctx, PFMP_ERR_ARG, "hmc: bad spec");
    if (sp->gauge_steps <= 0 || !(sp->tau > 0) || !(sp->tol > 0)) return set_err(ctx, PFMP_ERR_ARG, "hmc: bad spec");
    for (int j = 0; j < sp->nterms; j++) {
        const pfmp_term &t = sp->terms[j];
        if (t.steps <= 0 || t.op < 0 || t.op >= PFMP_MAX_OPS || !ctx->ops[t.op].valid)
            return set_err(ctx, PFMP_ERR_ARG, "hmc: term operator or steps");
        if (t.kind == PFMP_TERM_RATIO && (t.op2 < 0 || t.op2 >= PFMP_MAX_OPS || !ctx->ops[t.op2].valid))
            return set_err(ctx, PFMP_ERR_ARG, "hmc: ratio denominator");
        if ((t.kind == PFMP_TERM_POLY || t.kind == PFMP_TERM_POLYCORR || t.kind == PFMP_TERM_POLYQ) &&
            (t.n < 2 || (t.n & 1) || t.n + 1 > PFMP_MAX_SHIFTS))
            return set_err(ctx, PFMP_ERR_ARG, "hmc: polynomial degree must be even, 2..126");
        if (t.kind == PFMP_TERM_POLYQ && (t.n1 < 2 || (t.n1 & 1) || t.n1 >= t.n || (t.n + 1) % (t.n1 + 1)))
            return set_err(ctx, PFMP_ERR_ARG, "hmc: polyq needs an even n1 < n with (n1 + 1) dividing (n + 1)");
        if (t.kind < PFMP_TERM_POLY || t.kind > PFMP_TERM_POLYQ) return set_err(ctx, PFMP_ERR_ARG, "hmc: term kind");
    }
    return 0;
}

// The roots (in the order k = 1..n) and norm of a term's polynomial.  POLYQ: Q = P_n / P_n1
// has the roots of P_n whose angle 2 pi k / (n + 1) is not an angle 2 pi k' / (n1 + 1) of P_n1,
// i.e. k not a multiple of (n + 1) / (n1 + 1), and norm a_n / a_n1 (App. A).  In either case
// the first half of the list holds one root of each conjugate pair (k <= n / 2).
void roots_of(const pfmp_term &t, std::vector<cd> &z, double &a)
{
    std::vector<double> r(2 * t.n);
    double nm[2];
    pfmp_chebyshev(t.n, t.mu, t.nu, r.data(), nm);
    z.clear();
    const int m = t.kind == PFMP_TERM_POLYQ ? (t.n + 1) / (t.n1 + 1) : 0;
    for (int k = 1; k <= t.n; k++)
        if (m == 0 || k % m != 0) z.push_back(cd(r[2 * (k - 1)], r[2 * (k - 1) + 1]));
    a = nm[0];
    if (m) {
        std::vector<double> r1(2 * t.n1);
        double nm1[2];
        pfmp_chebyshev(t.n1, t.mu, t.nu, r1.data(), nm1);
        a /= nm1[0];
    }
}

// partial fractions: 1 / prod_k (x - z_k) = sum_i r_i / (x - z_i), r_i = prod_{j != i} 1 / (z_i - z_j)
std::vector<cd> residues(const std::vector<cd> &z)
{
    std::vector<cd> r(z.size());
    for (size_t i = 0; i < z.size(); i++) {
        cd p = 1.0;
        for (size_t j = 0; j < z.size(); j++)
            if (j != i) p /= (z[i] - z[j]);
        r[i] = p;
    }
    return r;
}

int partner(const std::vector<cd> &z, int i)
{
    int best = 0;
    for (size_t j = 0; j < z.size(); j++)
        if (std::abs(z[j] - std::conj(z[i])) < std::abs(z[best] - std::conj(z[i]))) best = (int)j;
    return best;
}

int solve(Ctx &X, int op, const void *b, void *x)
{
    pfmp_solver_params p{X.sp->tol, X.sp->maxiter > 0 ? X.sp->maxiter : 100000, X.sp->solver_prec, 0.0, 0};
    pfmp_solver_stats st{};
    int rc = X.sp->ptnet ? pfmp_fcg_solve(X.c, op, X.sp->ptnet, b, x, &p, &st) : pfmp_cg_solve(X.c, op, b, x, &p, &st);
    X.iters += st.iters;
    X.mhalf += 2 * st.kmults;
    return rc;
}

// the mixed-precision and learned modes (every solve to the same FP64 residual)
bool low_precision_mode(const Ctx &X) { return X.sp->solver_prec != PFMP_F64 || X.sp->ptnet; }

// x_k = (J - z_k)^-1 b for every pole.  The plain FP64 form runs all poles in one
// multi-shift solve.  In the mixed-precision and learned modes the pole z = 0, which
// needs the most iterations, is solved by that mode's CG (or taken from x0, solved
// beforehand with the other CG solves of the step), and the FP64 multi-shift solver
// stops as soon as the complex poles, well away from the spectrum, have converged.
int msolve(Ctx &X, int op, const std::vector<cd> &z, const void *b, std::vector<double2 *> &xs,
           const void *x0 = nullptr)
{
    int k0 = -1;
    if (low_precision_mode(X))
        for (size_t k = 0; k < z.size(); k++)
            if (z[k] == cd(0.0)) k0 = (int)k;
    std::vector<double> zz;
    std::vector<void *> xv;
    for (size_t k = 0; k < z.size(); k++) {
        if ((int)k == k0) continue;
        zz.push_back(z[k].real());
        zz.push_back(z[k].imag());
        xv.push_back(xs[k]);
    }
    int rc = 0;
    if (!xv.empty()) {
        pfmp_solver_params p{X.sp->tol, X.sp->maxiter > 0 ? X.sp->maxiter : 100000, PFMP_F64, 0.0, 0};
        pfmp_solver_stats st{};
        rc = pfmp_cg_multishift(X.c, op, (int)xv.size(), zz.data(), b, xv.data(), &p, &st);
        X.iters += st.iters;
        X.mhalf += 2 * st.kmults;
    }
    if (rc || k0 < 0) return rc;
    if (x0) {
        HIPCHK(X.c, hipMemcpyAsync(xs[k0], x0, sizeof(double) * spinor_reals(X.c->g), hipMemcpyDeviceToDevice,
                                   X.c->stream));
        return 0;
    }
    return solve(X, op, b, xs[k0]);
}

// Poles per multi-shift solve: each pole keeps its solution, its search direction and (for
// the force) its Mhat image, so the poles of a high-degree filter run in groups that fit
// kShiftBudget of device memory (a group of a large lattice, all poles at once on a small
// one).  A group holds whole conjugate pairs, which the force pairs up.  Every pole stops on
// its own residual, so its solution does not depend on the grouping.
constexpr double kShiftBudget = 48.0 * (1ull << 30);

std::vector<std::vector<int>> pole_groups(pfmp_ctx *ctx, const std::vector<cd> &z, bool pairs)
{
    const double vb = sizeof(double) * (double)spinor_reals(ctx->g);
    const int G = std::max(2, (int)std::min<double>(1e6, kShiftBudget / (3.0 * vb)));
    std::vector<std::vector<int>> groups(1);
    std::vector<bool> done(z.size(), false);
    for (size_t i = 0; i < z.size(); i++) {
        if (done[i]) continue;
        std::vector<int> mem{(int)i};
        done[i] = true;
        if (pairs) {
            const int j = partner(z, (int)i);
            if (!done[j]) {
                mem.push_back(j);
                done[j] = true;
            }
        }
        if ((int)(groups.back().size() + mem.size()) > G && !groups.back().empty()) groups.emplace_back();
        groups.back().insert(groups.back().end(), mem.begin(), mem.end());
    }
    return groups;
}

int applyM(Ctx &X, int op, int dag, const void *in, void *out, int prec = PFMP_F64)
{
    X.mhalf += 1;
    return pfmp_apply_M(X.c, op, dag, in, out, prec);
}

int poly(Ctx &X, int op, const std::vector<cd> &roots, cd norm, const void *in, void *out, void *const *chain,
         int prec = PFMP_F64)
{
    std::vector<double> r(2 * roots.size());
    for (size_t k = 0; k < roots.size(); k++) {
        r[2 * k] = roots[k].real();
        r[2 * k + 1] = roots[k].imag();
    }
    double nm[2] = {norm.real(), norm.imag()};
    X.mhalf += 2 * (long long)roots.size();
    return pfmp_apply_poly(X.c, op, (int)roots.size(), r.data(), nm, in, out, chain, prec);
}

cd dot(Ctx &X, const void *a, const void *b, int &rc)
{
    double d[2] = {0, 0};
    rc = pfmp_dot(X.c, a, b, d);
    return cd(d[0], d[1]);
}

// pool indices: [0,16) phi of pfmp_trajectory, [16, 32) temporaries, [32, ...) chains
constexpr int kTmp = 16, kChain = 32;

// S_j(phi)
int term_action(Ctx &X, const pfmp_term &t, const void *phi, double *S)
{
    pfmp_ctx *ctx = X.c;
    int rc = 0;
    double2 *t0 = pool_get(ctx, kTmp), *t1 = pool_get(ctx, kTmp + 1);
    if (!t0 || !t1) return set_err(ctx, PFMP_ERR_OOM, "hmc pool");
    switch (t.kind) {
    case PFMP_TERM_POLY:
    case PFMP_TERM_POLYQ: {
        std::vector<cd> z;
        double a;
        roots_of(t, z, a);
        if ((rc = poly(X, t.op, z, a, phi, t0, nullptr))) return rc;
        *S = dot(X, phi, t0, rc).real();
        return rc;
    }
    case PFMP_TERM_POLYCORR: {
        std::vector<cd> z;
        double a;
        roots_of(t, z, a);
        z.push_back(0.0);
        std::vector<cd> r = residues(z);
        cd s = 0;
        for (const std::vector<int> &grp : pole_groups(ctx, z, false)) {
            std::vector<cd> zg;
            std::vector<double2 *> xs;
            for (size_t q = 0; q < grp.size(); q++) {
                zg.push_back(z[grp[q]]);
                xs.push_back(pool_get(ctx, kChain + (int)q));
                if (!xs.back()) return set_err(ctx, PFMP_ERR_OOM, "hmc pool");
            }
            if ((rc = msolve(X, t.op, zg, phi, xs))) return rc;
            for (size_t q = 0; q < grp.size(); q++) {
                s += r[grp[q]] * dot(X, phi, xs[q], rc);
                if (rc) return rc;
            }
        }
        *S = (s / a).real();
        return 0;
    }
    case PFMP_TERM_RATIO:
        if ((rc = applyM(X, t.op, 0, phi, t0))) return rc;
        if ((rc = solve(X, t.op2, t0, t1))) return rc;
        *S = dot(X, t0, t1, rc).real();
        return rc;
    case PFMP_TERM_HEAVY:
        if ((rc = solve(X, t.op, phi, t0))) return rc;
        *S = dot(X, phi, t0, rc).real();
        return rc;
    }
    return set_err(ctx, PFMP_ERR_ARG, "hmc: unknown term");
}

int term_heatbath(Ctx &X, const pfmp_term &t, const void *eta, void *phi)
{
    pfmp_ctx *ctx = X.c;
    int rc = 0;
    double2 *t0 = pool_get(ctx, kTmp), *t1 = pool_get(ctx, kTmp + 1);
    if (!t0 || !t1) return set_err(ctx, PFMP_ERR_OOM, "hmc pool");
    switch (t.kind) {
    case PFMP_TERM_POLY:
    case PFMP_TERM_POLYQ: {
        // P = R^dag R, R = sqrt(a) prod (J - z_k) over the first half of the roots (one of
        // each conjugate pair); phi = R^-1 eta by partial fractions over those poles and
        // one multi-shift solve
        std::vector<cd> z;
        double a;
        roots_of(t, z, a);
        z.resize(z.size() / 2);
        std::vector<cd> r = residues(z);
        HIPCHK(ctx, hipMemsetAsync(phi, 0, sizeof(double) * spinor_reals(ctx->g), ctx->stream));
        for (const std::vector<int> &grp : pole_groups(ctx, z, false)) {
            std::vector<cd> zg;
            std::vector<double2 *> xs;
            for (size_t q = 0; q < grp.size(); q++) {
                zg.push_back(z[grp[q]]);
                xs.push_back(pool_get(ctx, kChain + (int)q));
                if (!xs.back()) return set_err(ctx, PFMP_ERR_OOM, "hmc pool");
            }
            if ((rc = msolve(X, t.op, zg, eta, xs))) return rc;
            for (size_t q = 0; q < grp.size(); q++) {
                cd c = r[grp[q]] / std::sqrt(a);
                double cc[2] = {c.real(), c.imag()}, one[2] = {1, 0};
                if ((rc = pfmp_axpby(ctx, cc, xs[q], one, phi))) return rc;
            }
        }
        return 0;
    }
    case PFMP_TERM_POLYCORR: {
        // phi = R^dag W^dag eta = sqrt(a) prod_{k<=n/2} (J - z_k^*) W^dag eta
        std::vector<cd> z;
        double a;
        roots_of(t, z, a);
        std::vector<cd> zc(t.n / 2);
        for (int k = 0; k < t.n / 2; k++) zc[k] = std::conj(z[k]);
        if ((rc = applyM(X, t.op, 1, eta, t0))) return rc;
        return poly(X, t.op, zc, std::sqrt(a), t0, phi, nullptr);
    }
    case PFMP_TERM_RATIO:
        // phi = J^-1 W^dag M_b^dag eta
        if ((rc = applyM(X, t.op2, 1, eta, t0))) return rc;
        if ((rc = applyM(X, t.op, 1, t0, t1))) return rc;
        return solve(X, t.op, t1, phi);
    case PFMP_TERM_HEAVY:
        return applyM(X, t.op, 1, eta, phi);
    }
    return set_err(ctx, PFMP_ERR_ARG, "hmc: unknown term");
}

// F += eps * dS_j/dw
int term_force(Ctx &X, const pfmp_term &t, const void *phi, double eps, double *F, const void *presolved = nullptr)
{
    pfmp_ctx *ctx = X.c;
    int rc = 0;
    std::vector<const void *> XX, YY;
    std::vector<double> cc;
    auto pair = [&](const void *x, const void *y, cd c) {
        XX.push_back(x);
        YY.push_back(y);
        cc.push_back(c.real());
        cc.push_back(c.imag());
    };
    switch (t.kind) {
    case PFMP_TERM_POLY:
    case PFMP_TERM_POLYQ: {
        std::vector<cd> z;
        double a;
        roots_of(t, z, a);
        const int n = (int)z.size();
        // chi_n..chi_1 from z_n..z_2 with norm a, all kept (C[k] = chi_{n-k}); eta_1 = phi and
        // eta_{i+1} = (J - z_i^*) eta_i formed one at a time as i runs up, with the Mhat images
        // of eta_i and chi_i and the force pairs of four i at a time in a ring of buffers: n + 12
        // vectors instead of 4n.  In the mixed-precision modes the chains, their Mhat images and
        // the force's odd-site intermediates are FP32 (FP32 links and clover); the force sums in
        // FP64 and the filter action stays FP64.
        const bool f32 = low_precision_mode(X);
        const int prec = f32 ? PFMP_F32 : PFMP_F64;
        constexpr int R = 4;
        std::vector<void *> C(n), E(R), WE(R), WC(R);
        for (int k = 0; k < n; k++)
            if (!(C[k] = pool_get(ctx, kChain + k))) return set_err(ctx, PFMP_ERR_OOM, "hmc pool");
        for (int q = 0; q < R; q++) {
            E[q] = pool_get(ctx, kChain + n + q);
            WE[q] = pool_get(ctx, kChain + n + R + q);
            WC[q] = pool_get(ctx, kChain + n + 2 * R + q);
            if (!E[q] || !WE[q] || !WC[q]) return set_err(ctx, PFMP_ERR_OOM, "hmc pool");
        }
        const void *src = phi;
        if (f32) {
            void *phi32 = pool_get(ctx, kChain + n + 3 * R);
            if (!phi32) return set_err(ctx, PFMP_ERR_OOM, "hmc pool");
            if ((rc = pfmp_convert_spinor(ctx, phi, PFMP_F64, phi32, PFMP_F32))) return rc;
            src = phi32;
        }
        std::vector<cd> rc_(n - 1);
        for (int k = 0; k < n - 1; k++) rc_[k] = z[n - 1 - k];
        if ((rc = poly(X, t.op, rc_, a, src, C[n - 1], C.data(), prec))) return rc;
        const void *eta = src;
        for (int i = 1; i <= n; i++) {
            const int q = (i - 1) % R;
            if (i > 1) {
                std::vector<cd> one{std::conj(z[i - 2])};
                if ((rc = poly(X, t.op, one, 1.0, eta, E[q], nullptr, prec))) return rc;
                eta = E[q];
            }
            const void *chi = C[n - i];
            if ((rc = applyM(X, t.op, 0, eta, WE[q], prec))) return rc;
            if ((rc = applyM(X, t.op, 0, chi, WC[q], prec))) return rc;
            pair(WE[q], chi, eps);
            pair(WC[q], eta, eps);
            if (q == R - 1 || i == n) {
                rc = f32 ? fermion_force_f32(ctx, t.op, (int)XX.size(), XX.data(), YY.data(), cc.data(), F)
                         : pfmp_fermion_force(ctx, t.op, (int)XX.size(), XX.data(), YY.data(), cc.data(), 0, F);
                if (rc) return rc;
                XX.clear();
                YY.clear();
                cc.clear();
            }
        }
        return 0;
    }
    case PFMP_TERM_POLYCORR: {
        std::vector<cd> z;
        double a;
        roots_of(t, z, a);
        z.push_back(0.0);
        std::vector<cd> r = residues(z);
        const auto groups = pole_groups(ctx, z, true);
        size_t G = 0;
        for (const auto &grp : groups) G = std::max(G, grp.size());
        for (const std::vector<int> &grp : groups) {
            const int m = (int)grp.size();
            std::vector<cd> zg(m);
            std::vector<double2 *> xs(m), wx(m);
            std::vector<int> slot(z.size(), -1);
            for (int q = 0; q < m; q++) {
                zg[q] = z[grp[q]];
                slot[grp[q]] = q;
                xs[q] = pool_get(ctx, kChain + q);
                wx[q] = pool_get(ctx, kChain + (int)G + q);
                if (!xs[q] || !wx[q]) return set_err(ctx, PFMP_ERR_OOM, "hmc pool");
            }
            // the pole z = 0 is the last one; a presolved x for it belongs to its group only
            const bool has0 = slot[z.size() - 1] >= 0;
            if ((rc = msolve(X, t.op, zg, phi, xs, has0 ? presolved : nullptr))) return rc;
            for (int q = 0; q < m; q++)
                if ((rc = applyM(X, t.op, 0, xs[q], wx[q]))) return rc;
            XX.clear();
            YY.clear();
            cc.clear();
            for (int q = 0; q < m; q++) {
                const int i = grp[q], j = slot[partner(z, i)];
                cd c = -eps * r[i] / a;
                // Re[c x_j^dag dJ x_i]
                pair(wx[j], xs[q], c);
                pair(wx[q], xs[j], std::conj(c));
            }
            if ((rc = pfmp_fermion_force(ctx, t.op, (int)XX.size(), XX.data(), YY.data(), cc.data(), 0, F)))
                return rc;
        }
        return 0;
    }
    case PFMP_TERM_RATIO: {
        double2 *t0 = pool_get(ctx, kTmp), *x = pool_get(ctx, kTmp + 1), *mx = pool_get(ctx, kTmp + 2);
        if (!t0 || !x || !mx) return set_err(ctx, PFMP_ERR_OOM, "hmc pool");
        if (presolved) {
            x = (double2 *)presolved;
        } else {
            if ((rc = applyM(X, t.op, 0, phi, t0))) return rc;
            if ((rc = solve(X, t.op2, t0, x))) return rc;
        }
        if ((rc = applyM(X, t.op2, 0, x, mx))) return rc;
        const void *xa[1] = {x}, *ya[1] = {phi};
        double ca[2] = {2 * eps, 0};
        if ((rc = pfmp_fermion_force(ctx, t.op, 1, xa, ya, ca, 0, F))) return rc;
        const void *xb[1] = {mx}, *yb[1] = {x};
        double cb[2] = {-2 * eps, 0};
        return pfmp_fermion_force(ctx, t.op2, 1, xb, yb, cb, 0, F);
    }
    case PFMP_TERM_HEAVY: {
        double2 *x = pool_get(ctx, kTmp + 1), *wx = pool_get(ctx, kTmp + 2);
        if (!x || !wx) return set_err(ctx, PFMP_ERR_OOM, "hmc pool");
        if (presolved) x = (double2 *)presolved;
        else if ((rc = solve(X, t.op, phi, x))) return rc;
        if ((rc = applyM(X, t.op, 0, x, wx))) return rc;
        const void *xa[1] = {wx}, *ya[1] = {x};
        double ca[2] = {-2 * eps, 0};
        return pfmp_fermion_force(ctx, t.op, 1, xa, ya, ca, 0, F);
    }
    }
    return set_err(ctx, PFMP_ERR_ARG, "hmc: unknown term");
}

int hamiltonian(Ctx &X, const double *P, const void *const *phi, double *parts, bool with_terms)
{
    pfmp_ctx *ctx = X.c;
    const pfmp_hmc_spec *sp = X.sp;
    int rc;
    if ((rc = pfmp_kinetic(ctx, P, &parts[0]))) return rc;
    if ((rc = pfmp_gauge_action(ctx, sp->beta, &parts[1]))) return rc;
    parts[2] = 0;
    if (sp->det_op >= 0 && (rc = pfmp_logdet_action(ctx, sp->det_op, &parts[2]))) return rc;
    if (with_terms)
        for (int j = 0; j < sp->nterms; j++)
            if ((rc = term_action(X, sp->terms[j], phi[j], &parts[3 + j]))) return rc;
    return 0;
}

}  // namespace

extern "C" int pfmp_heatbath(pfmp_ctx *ctx, const pfmp_hmc_spec *spec, const void *const *eta, void *const *phi)
{
    if (!ctx) return PFMP_ERR_ARG;
    int rc = chk_spec(ctx, spec);
    if (rc) return rc;
    if (spec->nterms > 0 && (!eta || !phi)) return set_err(ctx, PFMP_ERR_ARG, "heatbath: null buffers");
    Ctx X{ctx, spec};
    for (int j = 0; j < spec->nterms; j++)
        if ((rc = term_heatbath(X, spec->terms[j], eta[j], phi[j]))) return rc;
    return 0;
}

extern "C" int pfmp_hamiltonian(pfmp_ctx *ctx, const pfmp_hmc_spec *spec, const double *P, const void *const *phi,
                                double *H, double *parts)
{
    if (!ctx || !P || !H) return ctx ? set_err(ctx, PFMP_ERR_ARG, "hamiltonian: null") : PFMP_ERR_ARG;
    int rc = chk_spec(ctx, spec);
    if (rc) return rc;
    Ctx X{ctx, spec};
    double loc[PFMP_MAX_TERMS + 3] = {0};
    if ((rc = hamiltonian(X, P, phi, loc, true))) return rc;
    double s = 0;
    for (int k = 0; k < spec->nterms + 3; k++) s += loc[k];
    *H = s;
    if (parts) std::memcpy(parts, loc, sizeof(double) * (spec->nterms + 3));
    return 0;
}

extern "C" int pfmp_force_norms(pfmp_ctx *ctx, const pfmp_hmc_spec *spec, const void *const *phi, double *out)
{
    if (!ctx || !out || (spec && spec->nterms > 0 && !phi))
        return ctx ? set_err(ctx, PFMP_ERR_ARG, "force_norms: null") : PFMP_ERR_ARG;
    int rc = chk_spec(ctx, spec);
    if (rc) return rc;
    Ctx X{ctx, spec};
    double *F = (double *)ws_alloc(ctx, sizeof(double) * mom_reals(ctx->g), 24);
    if (!F) return set_err(ctx, PFMP_ERR_OOM, "force buffer");
    const int nrow = spec->nterms + 2;
    for (int r = 0; r < nrow; r++) {
        out[2 * r] = out[2 * r + 1] = 0;
        if (r == nrow - 1 && spec->det_op < 0) continue;
        HIPCHK(ctx, hipMemsetAsync(F, 0, sizeof(double) * mom_reals(ctx->g), ctx->stream));
        if (r == 0) rc = pfmp_gauge_force(ctx, spec->beta, F);
        else if (r < nrow - 1) rc = term_force(X, spec->terms[r - 1], phi[r - 1], 1.0, F);
        else rc = pfmp_logdet_force(ctx, spec->det_op, 1.0, F);
        if (rc || (rc = force_norms(ctx, F, &out[2 * r], &out[2 * r + 1]))) return rc;
    }
    return 0;
}

static int md_evolve(Ctx &X, double *P, const void *const *phi, pfmp_traj_stats *st)
{
    pfmp_ctx *ctx = X.c;
    const pfmp_hmc_spec *sp = X.sp;
    const int nt = sp->nterms + 1;
    const double lam = sp->lambda != 0 ? sp->lambda : kOmelyanLambda;
    // rows: gauge, the terms, and S_det on its own scale when det_steps > 0
    const bool det_row = sp->det_steps > 0 && sp->det_op >= 0;
    const int nrow = nt + (det_row ? 1 : 0);
    int64_t L = 2LL * sp->gauge_steps;
    for (int j = 0; j < sp->nterms; j++) L = lcm64(L, 2LL * sp->terms[j].steps);
    if (det_row) L = lcm64(L, 2LL * sp->det_steps);
    std::vector<Scheme> sch;
    sch.push_back(omelyan(sp->gauge_steps, L, sp->tau, lam));
    for (int j = 0; j < sp->nterms; j++) sch.push_back(omelyan(sp->terms[j].steps, L, sp->tau, lam));
    if (det_row) sch.push_back(omelyan(sp->det_steps, L, sp->tau, lam));
    std::vector<int> len(nrow);
    std::vector<int64_t> T;
    std::vector<double> S;
    int cap = 0;
    for (int j = 0; j < nrow; j++) {
        len[j] = (int)sch[j].T.size();
        cap += len[j];
        T.insert(T.end(), sch[j].T.begin(), sch[j].T.end());
        S.insert(S.end(), sch[j].S.begin(), sch[j].S.end());
    }
    std::vector<int64_t> To(cap);
    std::vector<double> So((size_t)cap * nrow);
    int nout = 0;
    int rc = pfmp_schedule_build(nrow, len.data(), T.data(), S.data(), cap, To.data(), So.data(), &nout);
    if (rc) return set_err(ctx, rc, "hmc: schedule merge failed");
    double *F = (double *)ws_alloc(ctx, sizeof(double) * mom_reals(ctx->g), 24);
    if (!F) return set_err(ctx, PFMP_ERR_OOM, "force buffer");
    const double tick = sp->tau / (double)L;
    const auto t_md = std::chrono::steady_clock::now();
    if (st) {
        st->nsteps = nout;
        for (int j = 0; j < nt; j++) st->nforce[j] = 0;
        st->nforce_det = 0;
    }
    // A merged step whose only force is the gauge force (the finest scale between fermion
    // force steps) is T then P -= eps F_G, with the gauge force added straight into P: the
    // coefficients of -F_G are exactly the negated coefficients of F_G, so this equals the
    // force buffer route bit for bit.  A run of such steps is replayed as one HIP graph
    // (keyed by its step sizes); the links' derived fields are marked stale after it.
    const bool det_on_gauge_row = sp->det_op >= 0 && !det_row;
    auto gauge_only = [&](int k) {
        if (So[k] == 0.0 || det_on_gauge_row) return false;
        for (int j = 1; j < nrow; j++)
            if (So[(size_t)j * cap + k] != 0.0) return false;
        return true;
    };
    for (int k = 0; k < nout; k++) {
        if (gauge_only(k)) {
            int k2 = k;
            while (k2 + 1 < nout && gauge_only(k2 + 1)) k2++;
            std::vector<uint64_t> key;
            key_add(key, 6);   // run of gauge-only merged steps
            key_geom(key, ctx->g);
            key_add(key, (const void *)ctx->U);
            key_add(key, (const void *)P);
            key_add(key, sp->beta);
            for (int q = k; q <= k2; q++) {
                key_add(key, tick * (double)To[q]);
                key_add(key, So[q]);
            }
            auto run = [&]() -> int {
                int e;
                for (int q = k; q <= k2; q++) {
                    if (To[q] != 0 && (e = pfmp_update_gauge(ctx, tick * (double)To[q], P))) return e;
                    if ((e = pfmp_gauge_force(ctx, -sp->beta * So[q], P))) return e;
                }
                return 0;
            };
            if ((rc = graph_run(ctx, key, 1, run))) return rc;
            if ((rc = rebuild_gauge_derived(ctx))) return rc;
            if (st) st->nforce[0] += k2 - k + 1;
            k = k2;
            continue;
        }
        if (To[k] != 0 && (rc = pfmp_update_gauge(ctx, tick * (double)To[k], P))) return rc;
        bool any = false;
        for (int j = 0; j < nrow; j++) any = any || So[(size_t)j * cap + k] != 0.0;
        if (!any) continue;
        HIPCHK(ctx, hipMemsetAsync(F, 0, sizeof(double) * mom_reals(ctx->g), ctx->stream));
        // the CG solves of the RATIO / HEAVY terms due at this step, as one multi-RHS solve
        std::vector<const void *> pre(nt, nullptr);
        if (sp->batch && !sp->ptnet) {
            std::vector<int> js, sops;
            std::vector<const void *> rhs;
            std::vector<void *> sol;
            for (int j = 1; j < nt; j++) {
                const pfmp_term &t = sp->terms[j - 1];
                // the correction term's z = 0 pole is a CG solve on J in the low-precision modes
                const bool pole0 = t.kind == PFMP_TERM_POLYCORR && low_precision_mode(X);
                if (So[(size_t)j * cap + k] == 0.0 ||
                    (t.kind != PFMP_TERM_RATIO && t.kind != PFMP_TERM_HEAVY && !pole0))
                    continue;
                double2 *b = pool_get(ctx, 2200 + j), *x = pool_get(ctx, 2100 + j);
                if (!b || !x) return set_err(ctx, PFMP_ERR_OOM, "hmc pool");
                if (t.kind == PFMP_TERM_RATIO) {
                    if ((rc = applyM(X, t.op, 0, phi[j - 1], b))) return rc;
                    rhs.push_back(b);
                    sops.push_back(t.op2);
                } else {
                    rhs.push_back(phi[j - 1]);
                    sops.push_back(t.op);
                }
                sol.push_back(x);
                js.push_back(j);
            }
            // one multi-RHS solve per group of operators of equal clover flag, at most 8 each
            for (int cl = 0; cl < 2; cl++) {
                std::vector<size_t> grp;
                for (size_t q = 0; q < js.size(); q++)
                    if ((ctx->ops[sops[q]].csw != 0) == (cl == 1)) grp.push_back(q);
                for (size_t g0 = 0; g0 < grp.size(); g0 += 8) {
                    size_t m = std::min<size_t>(8, grp.size() - g0);
                    std::vector<int> o(m);
                    std::vector<const void *> bb(m);
                    std::vector<void *> xx(m);
                    for (size_t q = 0; q < m; q++) {
                        o[q] = sops[grp[g0 + q]];
                        bb[q] = rhs[grp[g0 + q]];
                        xx[q] = sol[grp[g0 + q]];
                    }
                    if (m == 1) {
                        if ((rc = solve(X, o[0], bb[0], xx[0]))) return rc;
                    } else {
                        pfmp_solver_params p{sp->tol, sp->maxiter > 0 ? sp->maxiter : 100000, sp->solver_prec,
                                             0.0, 0};
                        std::vector<pfmp_solver_stats> bst(m);
                        if ((rc = pfmp_cg_solve_batch(ctx, (int)m, o.data(), bb.data(), xx.data(), &p, bst.data())))
                            return rc;
                        for (size_t q = 0; q < m; q++) {
                            X.iters += bst[q].iters;
                            X.mhalf += 2 * bst[q].kmults;
                        }
                    }
                    for (size_t q = 0; q < m; q++) pre[js[grp[g0 + q]]] = xx[q];
                }
            }
        }
        // the clover-force insertions of all terms due at this step go into one field,
        // applied by one clover-force pass before the momentum update
        struct DeferGuard {
            pfmp_ctx *c;
            ~DeferGuard()
            {
                c->clover_defer = false;
                c->phi_pending = false;
            }
        } guard{ctx};
        clover_force_defer(ctx);
        for (int j = 0; j < nt; j++) {
            double eps = So[(size_t)j * cap + k];
            if (eps == 0.0) continue;
            if (st) st->nforce[j]++;
            if (j == 0) {
                if ((rc = pfmp_gauge_force(ctx, sp->beta * eps, F))) return rc;
                if (sp->det_op >= 0 && !det_row && (rc = pfmp_logdet_force(ctx, sp->det_op, eps, F))) return rc;
            } else if ((rc = term_force(X, sp->terms[j - 1], phi[j - 1], eps, F, pre[j]))) {
                return rc;
            }
        }
        if (det_row) {
            double eps = So[(size_t)nt * cap + k];
            if (eps != 0.0) {
                if (st) st->nforce_det++;
                if ((rc = pfmp_logdet_force(ctx, sp->det_op, eps, F))) return rc;
            }
        }
        if ((rc = clover_force_flush(ctx, F))) return rc;
        if ((rc = pfmp_update_momenta(ctx, 1.0, F, P))) return rc;
        if (ctx->verbose) {
            std::string rows;
            for (int j = 0; j < nrow; j++)
                if (So[(size_t)j * cap + k] != 0.0) rows += (rows.empty() ? "" : ",") + std::to_string(j);
            std::fprintf(stderr, "[pfmp] md step %d/%d rows %s: %lld solver iterations so far, %.1f s\n", k + 1, nout,
                         rows.c_str(), X.iters,
                         std::chrono::duration<double>(std::chrono::steady_clock::now() - t_md).count());
            std::fflush(stderr);
        }
    }
    return 0;
}

extern "C" int pfmp_md_evolve(pfmp_ctx *ctx, const pfmp_hmc_spec *spec, double *P, const void *const *phi,
                              pfmp_traj_stats *st)
{
    if (!ctx || !P) return ctx ? set_err(ctx, PFMP_ERR_ARG, "md_evolve: null") : PFMP_ERR_ARG;
    int rc = chk_spec(ctx, spec);
    if (rc) return rc;
    Ctx X{ctx, spec};
    rc = md_evolve(X, P, phi, st);
    if (st) {
        st->kmults = X.mhalf / 2;
        st->solver_iters = X.iters;
    }
    return rc;
}

extern "C" int pfmp_trajectory(pfmp_ctx *ctx, const pfmp_hmc_spec *spec, const double *P0, const void *const *eta,
                               double u, double *P_end, pfmp_traj_stats *st)
{
    if (!ctx || !P0) return ctx ? set_err(ctx, PFMP_ERR_ARG, "trajectory: null") : PFMP_ERR_ARG;
    int rc = chk_spec(ctx, spec);
    if (rc) return rc;
    if (spec->nterms > 0 && !eta) return set_err(ctx, PFMP_ERR_ARG, "trajectory: null eta");
    auto t0 = std::chrono::steady_clock::now();
    Ctx X{ctx, spec};
    const Geom &g = ctx->g;
    size_t mb = sizeof(double) * mom_reals(g), gb = sizeof(double) * gauge_reals(g);
    double *P = (double *)ws_alloc(ctx, mb, 25);
    double2 *U0 = (double2 *)ws_alloc(ctx, gb, 26);
    if (!P || !U0) return set_err(ctx, PFMP_ERR_OOM, "trajectory buffers");
    HIPCHK(ctx, hipMemcpyAsync(P, P0, mb, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(U0, ctx->U, gb, hipMemcpyDeviceToDevice, ctx->stream));
    // Any failure from here on (a solve that hits maxiter, an allocation, a launch) puts the
    // start field back and marks everything derived from the links stale, so a caller that
    // catches the error goes on from the configuration it passed in.  The error text of the
    // failure is kept.
    struct Restore {
        pfmp_ctx *c;
        const double2 *U0;
        size_t gb;
        bool armed = true;
        void now()
        {
            armed = false;
            hipMemcpyAsync(c->U, U0, gb, hipMemcpyDeviceToDevice, c->stream);
            hipStreamSynchronize(c->stream);
            rebuild_gauge_derived(c);
        }
        ~Restore()
        {
            if (armed) now();
        }
    } restore{ctx, U0, gb};
    std::vector<void *> phi(spec->nterms);
    for (int j = 0; j < spec->nterms; j++)
        if (!(phi[j] = pool_get(ctx, j))) return set_err(ctx, PFMP_ERR_OOM, "hmc pool");
    auto phase = [&](const char *what) {
        if (!ctx->verbose) return;
        std::fprintf(stderr, "[pfmp] trajectory: %s, %lld solver iterations, %.1f s\n", what, X.iters,
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
        std::fflush(stderr);
    };
    for (int j = 0; j < spec->nterms; j++)
        if ((rc = term_heatbath(X, spec->terms[j], eta[j], phi[j]))) return rc;
    phase("heatbath done");
    double p0[PFMP_MAX_TERMS + 3] = {0}, p1[PFMP_MAX_TERMS + 3] = {0};
    if ((rc = hamiltonian(X, P, phi.data(), p0, spec->exact_start != 0))) return rc;
    phase("H0 done");
    if (!spec->exact_start)
        for (int j = 0; j < spec->nterms; j++) {
            p0[3 + j] = dot(X, eta[j], eta[j], rc).real();
            if (rc) return rc;
        }
    pfmp_traj_stats loc{};
    if ((rc = md_evolve(X, P, phi.data(), &loc))) return rc;
    phase("molecular dynamics done");
    if ((rc = hamiltonian(X, P, phi.data(), p1, true))) return rc;
    phase("H1 done");
    double H0 = 0, H1 = 0;
    for (int k = 0; k < spec->nterms + 3; k++) {
        H0 += p0[k];
        H1 += p1[k];
    }
    double dH = H1 - H0;
    int acc = (dH <= 0 || u < std::exp(-dH)) ? 1 : 0;
    if (P_end) HIPCHK(ctx, hipMemcpyAsync(P_end, P, mb, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    // accepted: keep the evolved links; rejected: back to the start field
    if (acc) restore.armed = false;
    else restore.now();
    auto t1 = std::chrono::steady_clock::now();
    if (st) {
        *st = loc;
        st->H0 = H0;
        st->H1 = H1;
        st->dH = dH;
        st->accept = acc;
        st->kmults = X.mhalf / 2;
        st->solver_iters = X.iters;
        st->seconds = std::chrono::duration<double>(t1 - t0).count();
        std::memcpy(st->parts0, p0, sizeof(p0));
        std::memcpy(st->parts1, p1, sizeof(p1));
    }
    return 0;
}
