/* Driver for the sanitizer build of the oracle (test infrastructure): runs
 * the oracle's 1D and 2D entry points on small seeded states under
 * AddressSanitizer and UndefinedBehaviorSanitizer.  The states come from a
 * plain linear congruential generator; nothing here computes the method. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dgref.h"

static uint64_t lcg = 88172645463325252ull;
static double unif(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * 0x1p-53;
}

static int run1d(int k, int filter, int pp, int bc)
{
    dgref_problem1d P;
    memset(&P, 0, sizeof P);
    P.eq = DGREF_EULER;
    P.k = k;
    P.filter = filter;
    P.bc[0] = P.bc[1] = bc;
    P.n = 37;
    P.lo = -1.0;
    P.hi = 1.0;
    P.gamma = 1.4;
    P.cfl = 0.1;
    P.pp = pp;
    for (int s = 0; s < 2; ++s)
        for (int v = 0; v < 3; ++v) P.dirichlet[s][v] = v == 2 ? 2.5 : (v == 0 ? 1.0 : 0.0);
    const int64_t n = P.n;
    double* u = calloc((size_t)3 * (k + 1) * n, sizeof(double));
    for (int64_t j = 0; j < n; ++j) {
        double rho = 0.5 + unif(), vel = unif() - 0.5, p = 0.2 + unif();
        u[(0 * (k + 1)) * n + j] = rho;
        u[(1 * (k + 1)) * n + j] = rho * vel;
        u[(2 * (k + 1)) * n + j] = p / 0.4 + 0.5 * rho * vel * vel;
        for (int v = 0; v < 3; ++v)
            for (int l = 1; l <= k; ++l) u[(v * (k + 1) + l) * n + j] = 0.05 * (unif() - 0.5);
    }
    dgref_report rep;
    int rc = dgref_run1d(&P, 1e30, 25, u, &rep);
    double* E = calloc((size_t)n * (k + 1), sizeof(double));
    double* eta = calloc((size_t)n, sizeof(double));
    dgref_exponents1d(&P, 1e-3, u, E, eta);
    free(E);
    free(eta);
    free(u);
    return rc;
}

static int run2d(int k, int filter, int pp, int basis, int reading)
{
    dgref_problem2d P;
    memset(&P, 0, sizeof P);
    P.eq = DGREF_EULER;
    P.k = k;
    P.filter = filter;
    P.bc[0] = DGREF_DIRICHLET;
    P.bc[1] = DGREF_OUTFLOW;
    P.bc[2] = 4;
    P.bc[3] = 5;
    P.nx = 13;
    P.ny = 7;
    P.xhi = 4.0;
    P.yhi = 1.0;
    P.gamma = 1.4;
    P.cfl = 0.1;
    P.pp = pp;
    P.basis = basis;
    P.cf_reading = reading;
    P.shock_x0 = 0.5;
    P.shock_speed = 3.0;
    const double post[4] = {2.0, 1.0, -0.5, 8.0}, pre[4] = {1.0, 0.0, 0.0, 2.5};
    for (int v = 0; v < 4; ++v) {
        P.post[v] = post[v];
        P.pre[v] = pre[v];
        for (int s = 0; s < 4; ++s) P.dirichlet[s][v] = post[v];
    }
    const int nm = (k + 1) * (k + 1);
    const int64_t nc = P.nx * P.ny;
    double* u = calloc((size_t)4 * nm * nc, sizeof(double));
    for (int64_t c = 0; c < nc; ++c) {
        const double* st = (c % P.nx) < 4 ? post : pre;
        for (int v = 0; v < 4; ++v) {
            u[(size_t)(v * nm) * nc + c] = st[v];
            for (int m = 1; m < nm; ++m)
                u[(size_t)(v * nm + m) * nc + c] = 0.02 * st[0] * (unif() - 0.5);
        }
    }
    dgref_report rep;
    int rc = dgref_run2d(&P, 1e30, 6, u, &rep);
    double* E = calloc((size_t)nc * (2 * k + 1), sizeof(double));
    double* eta = calloc((size_t)nc, sizeof(double));
    dgref_exponents2d(&P, 0.0, 1e-3, u, E, eta);
    double xi[6 * 8 + 64], et[6 * 8 + 64];
    dgref_pp_points2d(&P, xi, et);
    free(E);
    free(eta);
    free(u);
    return rc;
}

int main(void)
{
    int bad = 0;
    for (int k = 0; k <= 3; ++k)
        for (int filter = 0; filter <= 2; ++filter)
            for (int bc = 0; bc <= 3; ++bc) {
                const int rc = run1d(k, filter, k > 0, bc);
                if (rc != 0 && rc != DGREF_ERR_POSITIVITY) ++bad;
            }
    for (int k = 0; k <= 3; ++k)
        for (int filter = 0; filter <= 2; ++filter)
            for (int basis = 0; basis <= 1; ++basis) {
                const int rc = run2d(k, filter, 1, basis, (k + filter) % 3);
                if (rc != 0 && rc != DGREF_ERR_POSITIVITY) ++bad;
            }
    printf("sanitized oracle driver: %d unexpected return codes\n", bad);
    return bad ? 1 : 0;
}
