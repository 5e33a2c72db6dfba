// host.cpp -- host-side scalars of the method: Chebyshev roots and normalisation
// (paper App. A) and the generalized multi-scale schedule merge (App. B).
#include <cmath>
#include <complex>
#include <cstdint>
#include <vector>

#include "pfmp.h"

extern "C" int pfmp_chebyshev(int n, double mu, double nu, double *roots, double norm[2])
{
    if (n < 0 || !(mu >= nu) || !(nu > 0) || (n > 0 && !roots) || !norm) return PFMP_ERR_ARG;
    const double b = std::sqrt(mu * mu - nu * nu);
    std::complex<double> prod(mu, 0.0);
    for (int k = 1; k <= n; k++) {
        const double th = 2.0 * M_PI * k / (n + 1);
        std::complex<double> z(mu * (1.0 - std::cos(th)), -b * std::sin(th));
        roots[2 * (k - 1)] = z.real();
        roots[2 * (k - 1) + 1] = z.imag();
        prod *= (mu - z);
    }
    std::complex<double> a = 1.0 / prod;
    norm[0] = a.real();
    norm[1] = a.imag();
    return 0;
}

// Time-step insertion: advance by the smallest pending time step of all schemes;
// schemes whose pending step ends there contribute their next space step, the
// others a zero space step and a shortened pending step.  Integer ticks make
// coincident insertion times exact.
extern "C" int pfmp_schedule_build(int nterms, const int *len, const int64_t *T_ticks, const double *S_steps,
                                   int cap, int64_t *T_out, double *S_out, int *nout)
{
    if (nterms <= 0 || !len || !T_ticks || !S_steps || !T_out || !S_out || !nout || cap <= 0) return PFMP_ERR_ARG;
    std::vector<long> off(nterms + 1, 0);
    for (int j = 0; j < nterms; j++) {
        if (len[j] <= 0) return PFMP_ERR_ARG;
        off[j + 1] = off[j] + len[j];
    }
    int64_t total = -1;
    for (int j = 0; j < nterms; j++) {
        int64_t s = 0;
        for (long k = off[j]; k < off[j + 1]; k++) {
            if (T_ticks[k] < 0) return PFMP_ERR_ARG;
            s += T_ticks[k];
        }
        if (total >= 0 && s != total) return PFMP_ERR_ARG;
        total = s;
    }
    std::vector<long> head(nterms);
    std::vector<int64_t> pending(nterms);
    for (int j = 0; j < nterms; j++) {
        head[j] = off[j];
        pending[j] = T_ticks[off[j]];
    }
    int m = 0;
    int64_t tau = 0;
    bool first = true;
    while (first || tau < total) {
        first = false;
        int64_t d = INT64_MAX;
        for (int j = 0; j < nterms; j++) {
            if (head[j] >= off[j + 1]) return PFMP_ERR_ARG;
            if (pending[j] < d) d = pending[j];
        }
        if (m >= cap) return PFMP_ERR_ARG;
        T_out[m] = d;
        for (int j = 0; j < nterms; j++) {
            if (pending[j] == d) {
                S_out[(long)j * cap + m] = S_steps[head[j]];
                head[j]++;
                pending[j] = head[j] < off[j + 1] ? T_ticks[head[j]] : 0;
            } else {
                S_out[(long)j * cap + m] = 0.0;
                pending[j] -= d;
            }
        }
        tau += d;
        m++;
    }
    for (int j = 0; j < nterms; j++)
        if (head[j] != off[j + 1]) return PFMP_ERR_ARG;
    *nout = m;
    return 0;
}
