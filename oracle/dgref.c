/*
 * dgref.c — FP64 CPU oracle for the RKDG scheme with the jump filter
 * (arXiv:2407.19169).  TEST INFRASTRUCTURE ONLY: the plain, slow reference
 * the GPU library is checked against.  Nothing in the product path may load
 * it; it shares no code, header or table generator with the GPU library.
 *
 * Every formula is written out in the paper's own form (the damping
 * coefficient is built from c_f^l, the jump sums and (2/h)^2 l(l+1) exactly
 * as stated, not from a simplified closed form), with plain cell loops.
 * Readings of points the paper leaves open are marked "Reading:".
 */
#include "dgref.h"
#include "dgref_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif


/* ------------------------------------------------------------------------ */
/* Legendre polynomials and Gauss–Legendre quadrature                       */
/* ------------------------------------------------------------------------ */

/* Monomial coefficients of P_0..P_kmax from the three-term recurrence
 * (l+1) P_{l+1} = (2l+1) x P_l - l P_{l-1}. c[l][i] multiplies x^i.
 * Tables are evaluated in extended precision (long double) and rounded
 * once, so every tabulated value is the correctly rounded double. */
static void legendre_coeffs(int kmax, long double c[][MAXQ + 2])
{
    memset(c, 0, sizeof(long double) * (size_t)(kmax + 1) * (MAXQ + 2));
    c[0][0] = 1.0L;
    if (kmax >= 1) c[1][1] = 1.0L;
    for (int l = 1; l < kmax; ++l)
        for (int i = 0; i <= l + 1; ++i) {
            long double a = (i >= 1) ? (2.0L * l + 1.0L) * c[l][i - 1] : 0.0L;
            c[l + 1][i] = (a - l * c[l - 1][i]) / (l + 1.0L);
        }
}

static long double legendre_deriv_ld(int l, int m, long double xi)
{
    long double c[MAXQ + 2][MAXQ + 2];
    legendre_coeffs(l < 1 ? 1 : l, c);
    long double d[MAXQ + 2];
    for (int i = 0; i <= l; ++i) d[i] = c[l][i];
    for (int r = 0; r < m; ++r) /* differentiate m times */
        for (int i = 0; i <= l; ++i) d[i] = (i + 1 <= l) ? (i + 1) * d[i + 1] : 0.0L;
    long double s = 0.0L;
    for (int i = l; i >= 0; --i) s = s * xi + d[i];
    return s;
}

double dgref_legendre_deriv(int l, int m, double xi)
{
    if (l < 0 || l > MAXQ || m < 0) return NAN;
    return (double)legendre_deriv_ld(l, m, (long double)xi);
}

/* Gauss–Legendre nodes and weights by Newton's method on P_q (extended
 * precision), with P_q and P_{q-1} from the three-term recurrence and
 * P_q'(z) = q (z P_q - P_{q-1}) / (z^2 - 1),  w = 2 / ((1 - z^2) P_q'(z)^2). */
static void legendre_pair(int q, long double z, long double* pq, long double* pqm1)
{
    long double p0 = 1.0L, p1 = z;
    for (int l = 1; l < q; ++l) {
        long double p2 = ((2.0L * l + 1.0L) * z * p1 - l * p0) / (l + 1.0L);
        p0 = p1;
        p1 = p2;
    }
    *pq = p1;
    *pqm1 = p0;
}

static void gauss_ld(int q, long double* x, long double* w)
{
    for (int i = 0; i < q; ++i) {
        long double z = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (q + 0.5L));
        long double pq, pm1, dpq;
        for (int it = 0; it < 100; ++it) {
            legendre_pair(q, z, &pq, &pm1);
            dpq = q * (z * pq - pm1) / (z * z - 1.0L);
            long double dz = pq / dpq;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        legendre_pair(q, z, &pq, &pm1);
        dpq = q * (z * pq - pm1) / (z * z - 1.0L);
        x[q - 1 - i] = z; /* ascending order */
        w[q - 1 - i] = 2.0L / ((1.0L - z * z) * dpq * dpq);
    }
    if (q % 2 == 1) x[q / 2] = 0.0L; /* the middle node is exactly 0 */
}

int dgref_gauss(int q, double* x, double* w)
{
    if (q < 1 || q > MAXQ) return DGREF_ERR_ARG;
    long double xl[MAXQ], wl[MAXQ];
    gauss_ld(q, xl, wl);
    for (int i = 0; i < q; ++i) {
        x[i] = (double)xl[i];
        w[i] = (double)wl[i];
    }
    return DGREF_OK;
}

int dgref_make_basis(int k, int nq, dgref_basis* B)
{
    if (k < 0 || k > MAXK) return DGREF_ERR_ARG;
    if (nq == 0) nq = k + 1;
    if (nq < 1 || nq > MAXQ) return DGREF_ERR_ARG;
    B->k = k;
    B->nq = nq;
    long double xl[MAXQ], wl[MAXQ];
    gauss_ld(nq, xl, wl);
    for (int q = 0; q < nq; ++q) {
        B->xq[q] = (double)xl[q];
        B->wq[q] = (double)wl[q];
        for (int l = 0; l <= k; ++l) {
            B->phi[q][l] = (double)legendre_deriv_ld(l, 0, xl[q]);
            B->dphi[q][l] = (double)legendre_deriv_ld(l, 1, xl[q]);
        }
    }
    for (int s = 0; s < 2; ++s)
        for (int l = 0; l <= k; ++l)
            for (int m = 0; m <= k; ++m)
                B->tr[s][l][m] = dgref_legendre_deriv(l, m, s ? 1.0 : -1.0);
    return DGREF_OK;
}

/* The quadrature tables the oracle works with: nodes, weights, and
 * P_l, P_l' at the nodes (phi[q*(k+1)+l]). */
int dgref_basis_tables(int k, int nq, double* x, double* w, double* phi, double* dphi)
{
    dgref_basis B;
    int rc = dgref_make_basis(k, nq, &B);
    if (rc) return rc;
    for (int q = 0; q < B.nq; ++q) {
        x[q] = B.xq[q];
        w[q] = B.wq[q];
        for (int l = 0; l <= k; ++l) {
            phi[q * (k + 1) + l] = B.phi[q][l];
            dphi[q * (k + 1) + l] = B.dphi[q][l];
        }
    }
    return DGREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Physical fluxes                                                          */
/* ------------------------------------------------------------------------ */

int dgref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void dgref_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int dgref_nvars(int eq, int dim)
{
    if (eq == DGREF_EULER) return dim == 1 ? 3 : 4;
    return 1;
}

/* 1D flux f(u) (Sec. 3.1: Burgers f = u^2/2; Euler F(U) for U=(rho,m,E)). */
static void flux1d(int eq, double gamma, double a, const double* u, double* f)
{
    if (eq == DGREF_ADVECTION) {
        f[0] = a * u[0];
    } else if (eq == DGREF_BURGERS) {
        f[0] = 0.5 * u[0] * u[0];
    } else {
        double rho = u[0], m = u[1], E = u[2];
        double vel = m / rho;
        double p = (gamma - 1.0) * (E - 0.5 * m * vel);
        f[0] = m;
        f[1] = m * vel + p;
        f[2] = vel * (E + p);
    }
}

/* Largest characteristic speed |f'(u)| (Euler: |u| + c). */
static double lambda1d(int eq, double gamma, double a, const double* u)
{
    if (eq == DGREF_ADVECTION) return fabs(a);
    if (eq == DGREF_BURGERS) return fabs(u[0]);
    double rho = u[0], m = u[1], E = u[2];
    double vel = m / rho;
    double p = (gamma - 1.0) * (E - 0.5 * m * vel);
    return fabs(vel) + sqrt(gamma * p / rho);
}

/* Average enthalpy H = (E + p)/rho of the cell-average state (Euler only;
 * Reading: H-bar is evaluated at the cell-average conserved state). */
static double enthalpy1d(int eq, double gamma, const double* u)
{
    if (eq != DGREF_EULER) return 1.0;
    double rho = u[0], m = u[1], E = u[2];
    double p = (gamma - 1.0) * (E - 0.5 * m * m / rho);
    return (E + p) / rho;
}

/* Local Lax–Friedrichs flux (Sec. 3, named for all tests; the standard
 * two-point form with the larger of the two one-sided wave speeds). */
static void llf1d(int eq, double gamma, double a, const double* ul, const double* ur,
                  double* fh)
{
    int nv = dgref_nvars(eq, 1);
    double fl[MAXV], fr[MAXV];
    flux1d(eq, gamma, a, ul, fl);
    flux1d(eq, gamma, a, ur, fr);
    double al = lambda1d(eq, gamma, a, ul);
    double ar = lambda1d(eq, gamma, a, ur);
    double alpha = al > ar ? al : ar;
    for (int v = 0; v < nv; ++v) fh[v] = 0.5 * (fl[v] + fr[v]) - 0.5 * alpha * (ur[v] - ul[v]);
}

/* The interface flux the problem asks for: LLF, or HLL / HLLC (Euler). */
static void numflux1d(const dgref_problem1d* P, const double* ul, const double* ur, double* fh)
{
    if (P->eq == DGREF_EULER && P->flux != DGREF_FLUX_LLF)
        dgref_hll_flux(P->flux, 3, 0, P->gamma, ul, ur, fh);
    else
        llf1d(P->eq, P->gamma, P->adv_speed, ul, ur, fh);
}

int dgref_numflux1d(const dgref_problem1d* P, const double* ul, const double* ur, double* fh)
{
    if (!P || P->flux < DGREF_FLUX_LLF || P->flux > DGREF_FLUX_HLLC) return DGREF_ERR_ARG;
    numflux1d(P, ul, ur, fh);
    return DGREF_OK;
}

/* ------------------------------------------------------------------------ */
/* 1D helpers                                                               */
/* ------------------------------------------------------------------------ */

#define U1(u, v, l, j) ((u)[((size_t)(v) * (size_t)(K1) + (size_t)(l)) * (size_t)n + (size_t)(j)])

static int check1d(const dgref_problem1d* P)
{
    if (!P || P->n < 1 || P->k < 0 || P->k > MAXK) return DGREF_ERR_ARG;
    if (P->eq < 0 || P->eq > 2) return DGREF_ERR_ARG;
    if (!(P->hi > P->lo)) return DGREF_ERR_ARG;
    for (int s = 0; s < 2; ++s) {
        if (P->bc[s] < 0 || P->bc[s] > 3) return DGREF_ERR_ARG;
        if (P->bc[s] == DGREF_REFLECT && P->eq != DGREF_EULER) return DGREF_ERR_ARG;
    }
    if ((P->bc[0] == DGREF_PERIODIC) != (P->bc[1] == DGREF_PERIODIC)) return DGREF_ERR_ARG;
    return DGREF_OK;
}

/* m-th x-derivative of cell j's polynomial at its left (side 0) or right
 * (side 1) end: (2/h)^m sum_l u^l P_l^(m)(-1 / +1). */
static void trace1d(const dgref_problem1d* P, const dgref_basis* B, const double* u, int64_t j,
                    int side, int m, double h, double* out)
{
    const int K1 = P->k + 1;
    const int64_t n = P->n;
    int nv = dgref_nvars(P->eq, 1);
    double scale = pow(2.0 / h, m);
    for (int v = 0; v < nv; ++v) {
        double s = 0.0;
        for (int l = 0; l <= P->k; ++l) s += U1(u, v, l, j) * B->tr[side][l][m];
        out[v] = scale * s;
    }
}

/* Ghost value of the m-th derivative outside boundary `side` (0 = left end
 * of the domain, 1 = right end) given the interior one-sided value.
 * Reading of the boundary treatment: outflow copies the interior trace,
 * reflection mirrors it (momentum odd, the m-th derivative picks up
 * (-1)^m), Dirichlet is the prescribed constant state. */
static void ghost1d(const dgref_problem1d* P, int side, int m, const double* inner, double* g)
{
    int nv = dgref_nvars(P->eq, 1);
    int bc = P->bc[side];
    for (int v = 0; v < nv; ++v) {
        if (bc == DGREF_OUTFLOW) {
            g[v] = inner[v];
        } else if (bc == DGREF_REFLECT) {
            double sgn = (m % 2) ? -1.0 : 1.0;
            if (v == 1) sgn = -sgn;
            g[v] = sgn * inner[v];
        } else { /* Dirichlet */
            g[v] = (m == 0) ? P->dirichlet[side][v] : 0.0;
        }
    }
}

/* Left/right values of the m-th derivative at interface i (0..n), i.e. at
 * x_{i-1/2} between cells i-1 and i (0-based cells). */
static void iface1d(const dgref_problem1d* P, const dgref_basis* B, const double* u, int64_t i,
                    int m, double h, double* left, double* right)
{
    const int64_t n = P->n;
    if (i == 0) {
        trace1d(P, B, u, 0, 0, m, h, right);
        if (P->bc[0] == DGREF_PERIODIC)
            trace1d(P, B, u, n - 1, 1, m, h, left);
        else
            ghost1d(P, 0, m, right, left);
    } else if (i == n) {
        trace1d(P, B, u, n - 1, 1, m, h, left);
        if (P->bc[1] == DGREF_PERIODIC)
            trace1d(P, B, u, 0, 0, m, h, right);
        else
            ghost1d(P, 1, m, left, right);
    } else {
        trace1d(P, B, u, i - 1, 1, m, h, left);
        trace1d(P, B, u, i, 0, m, h, right);
    }
}

static void average1d(const dgref_problem1d* P, const double* u, int64_t j, double* ubar)
{
    const int K1 = P->k + 1;
    const int64_t n = P->n;
    int nv = dgref_nvars(P->eq, 1);
    for (int v = 0; v < nv; ++v) ubar[v] = U1(u, v, 0, j);
}

/* ------------------------------------------------------------------------ */
/* 1D semi-discrete DG operator (Sec. 2.1, scheme (scheme:DG))              */
/* ------------------------------------------------------------------------ */

/* L = du/dt of the semi-discrete scheme with v = P_l(xi):
 *   (h/(2l+1)) du^l/dt = int_{-1}^{1} f(u_h) P_l'(xi) dxi
 *                        - fhat_{j+1/2} P_l(1) + fhat_{j-1/2} P_l(-1).
 * The volume integral uses the Gauss rule of B.  fhat (nullable) receives
 * the interface fluxes, fhat[v*(n+1) + i]. */
int dgref_residual1d(const dgref_problem1d* P, const double* u, double* L, double* fhat)
{
    int rc = check1d(P);
    if (rc) return rc;
    dgref_basis B;
    if ((rc = dgref_make_basis(P->k, P->nq, &B))) return rc;
    const int K1 = P->k + 1;
    const int64_t n = P->n;
    const int nv = dgref_nvars(P->eq, 1);
    const double h = (P->hi - P->lo) / (double)n;

    double* fh = (double*)malloc(sizeof(double) * (size_t)nv * (size_t)(n + 1));
    if (!fh) return DGREF_ERR_ARG;

#pragma omp parallel for schedule(static) if (n >= 4096)
    for (int64_t i = 0; i <= n; ++i) {
        double ul[MAXV], ur[MAXV], f[MAXV];
        iface1d(P, &B, u, i, 0, h, ul, ur);
        numflux1d(P, ul, ur, f);
        for (int v = 0; v < nv; ++v) fh[(size_t)v * (size_t)(n + 1) + (size_t)i] = f[v];
    }

#pragma omp parallel for schedule(static) if (n >= 4096)
    for (int64_t j = 0; j < n; ++j) {
        double fq[MAXQ][MAXV];
        for (int q = 0; q < B.nq; ++q) {
            double uq[MAXV];
            for (int v = 0; v < nv; ++v) {
                double s = 0.0;
                for (int l = 0; l <= P->k; ++l) s += U1(u, v, l, j) * B.phi[q][l];
                uq[v] = s;
            }
            flux1d(P->eq, P->gamma, P->adv_speed, uq, fq[q]);
        }
        for (int v = 0; v < nv; ++v)
            for (int l = 0; l <= P->k; ++l) {
                double vol = 0.0;
                for (int q = 0; q < B.nq; ++q) vol += B.wq[q] * fq[q][v] * B.dphi[q][l];
                double fr = fh[(size_t)v * (size_t)(n + 1) + (size_t)(j + 1)];
                double fl = fh[(size_t)v * (size_t)(n + 1) + (size_t)j];
                double mass = h / (2.0 * l + 1.0);
                U1(L, v, l, j) = (vol - fr * B.tr[1][l][0] + fl * B.tr[0][l][0]) / mass;
            }
    }
    if (fhat) memcpy(fhat, fh, sizeof(double) * (size_t)nv * (size_t)(n + 1));
    free(fh);
    return DGREF_OK;
}

/* CFL wave speed: the largest |f'(u)| over the cell averages.
 * Reading: the paper only requires tau <= gamma h (Theorem 2.1); the
 * estimate from cell averages is the same quantity as beta_j. */
double dgref_max_wavespeed1d(const dgref_problem1d* P, const double* u)
{
    if (check1d(P)) return NAN;
    double amax = 0.0;
    for (int64_t j = 0; j < P->n; ++j) {
        double ub[MAXV];
        average1d(P, u, j, ub);
        double a = lambda1d(P->eq, P->gamma, P->adv_speed, ub);
        if (!(a <= amax)) amax = a; /* propagates NaN */
    }
    return amax;
}

/* SSP-RK3 in Shu–Osher form (Sec. 3, third-order SSP-RK; general form
 * (rkdg1)), without the post-stage filter:
 *   stage 0: u1  = un + dt L(un)
 *   stage 1: u2  = 3/4 un + 1/4 (u1 + dt L(u1))
 *   stage 2: un+1 = 1/3 un + 2/3 (u2 + dt L(u2))                          */
int dgref_stage1d(const dgref_problem1d* P, int stage, double dt, const double* un,
                  const double* us, double* out, double* fhat)
{
    int rc = check1d(P);
    if (rc) return rc;
    if (stage < 0 || stage > 2) return DGREF_ERR_ARG;
    const int nv = dgref_nvars(P->eq, 1);
    const size_t ndof = (size_t)nv * (size_t)(P->k + 1) * (size_t)P->n;
    const double* src = (stage == 0) ? un : us;
    double* L = (double*)malloc(sizeof(double) * ndof);
    if (!L) return DGREF_ERR_ARG;
    rc = dgref_residual1d(P, src, L, fhat);
    if (!rc) {
        for (size_t i = 0; i < ndof; ++i) {
            double adv = src[i] + dt * L[i];
            if (stage == 0)
                out[i] = adv;
            else if (stage == 1)
                out[i] = 0.75 * un[i] + 0.25 * adv;
            else
                out[i] = un[i] / 3.0 + 2.0 * adv / 3.0;
        }
    }
    free(L);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* 1D jump filter (Sec. 2.1 (para:damp2)-(para:damp21); systems Sec. 2.4    */
/* (para:dampsystems1d); Euler parameter c_f^l = beta/(4l(l+1)) / H-bar)    */
/* ------------------------------------------------------------------------ */

/* Damping exponents E[j*(k+1)+l] = sigma_j^l * dt for l = 0..k (E[.,0] = 0),
 * and the hybrid jump indicator eta_j = ||[u]||_{dK_j} / (2 h_j) (max over
 * components; Algorithm 1).  Jumps are taken from v, the unfiltered stage
 * output of all cells. */
int dgref_exponents1d(const dgref_problem1d* P, double dt, const double* v, double* E,
                      double* eta)
{
    int rc = check1d(P);
    if (rc) return rc;
    dgref_basis B;
    if ((rc = dgref_make_basis(P->k, P->nq, &B))) return rc;
    const int k = P->k;
    const int64_t n = P->n;
    const int nv = dgref_nvars(P->eq, 1);
    const double h = (P->hi - P->lo) / (double)n;

    /* |[d^m u]| at every interface: jmp[(i*(k+1) + m)*nv + var] */
    double* jmp = (double*)malloc(sizeof(double) * (size_t)(n + 1) * (size_t)(k + 1) * nv);
    if (!jmp) return DGREF_ERR_ARG;
#pragma omp parallel for schedule(static) if (n >= 4096)
    for (int64_t i = 0; i <= n; ++i)
        for (int m = 0; m <= k; ++m) {
            double a[MAXV], b[MAXV];
            iface1d(P, &B, v, i, m, h, a, b);
            for (int s = 0; s < nv; ++s)
                jmp[((size_t)i * (size_t)(k + 1) + (size_t)m) * nv + s] = fabs(b[s] - a[s]);
        }

#pragma omp parallel for schedule(static) if (n >= 4096)
    for (int64_t j = 0; j < n; ++j) {
        /* ||[d^m u^(s)]||_{dK_j}: sum of the two interface jumps */
        double J[MAXK + 1][MAXV];
        for (int m = 0; m <= k; ++m)
            for (int s = 0; s < nv; ++s)
                J[m][s] = jmp[((size_t)j * (size_t)(k + 1) + (size_t)m) * nv + s] +
                          jmp[((size_t)(j + 1) * (size_t)(k + 1) + (size_t)m) * nv + s];
        double ub[MAXV];
        average1d(P, v, j, ub);
        double beta = lambda1d(P->eq, P->gamma, P->adv_speed, ub); /* |f'(u-bar_j)| */
        double Hbar = enthalpy1d(P->eq, P->gamma, ub);
        E[(size_t)j * (size_t)(k + 1)] = 0.0; /* sigma^0 = 0: mode 0 is kept */
        for (int l = 1; l <= k; ++l) {
            double cf = beta / (4.0 * l * (l + 1.0)) / Hbar;
            double sig = 0.0; /* max over components of sigma_{j,l}(u^(s)) */
            for (int s = 0; s < nv; ++s) {
                double acc = h * J[0][s];
                for (int m = 1; m <= l; ++m) acc += m * (m + 1.0) * pow(h, m + 1) * J[m][s];
                double sjl = cf * acc;
                if (s == 0 || sjl > sig) sig = sjl;
            }
            double sigma_l = sig * (2.0 / h) * (2.0 / h) * l * (l + 1.0);
            E[(size_t)j * (size_t)(k + 1) + (size_t)l] = sigma_l * dt;
        }
        if (eta) {
            double e = 0.0;
            for (int s = 0; s < nv; ++s) {
                double es = J[0][s] / (2.0 * h);
                if (s == 0 || es > e) e = es;
            }
            eta[j] = e;
        }
    }
    free(jmp);
    return DGREF_OK;
}

/* u_j^l <- exp(-sigma_j^l dt) u_j^l (time-split solution (timespli:sys)). */
int dgref_filter1d(const dgref_problem1d* P, double dt, const double* v, double* out)
{
    int rc = check1d(P);
    if (rc) return rc;
    const int K1 = P->k + 1;
    const int64_t n = P->n;
    const int nv = dgref_nvars(P->eq, 1);
    double* E = (double*)malloc(sizeof(double) * (size_t)n * (size_t)K1);
    if (!E) return DGREF_ERR_ARG;
    rc = dgref_exponents1d(P, dt, v, E, NULL);
    if (!rc)
        for (int s = 0; s < nv; ++s)
            for (int l = 0; l < K1; ++l)
                for (int64_t j = 0; j < n; ++j)
                    U1(out, s, l, j) = exp(-E[(size_t)j * K1 + l]) * U1(v, s, l, j);
    free(E);
    return rc;
}

/* Hybrid procedure (Algorithm 1) with the jump filter as the low-order
 * limiter: troubled cells (eta_j > 1) get
 *   u_hyd = omega_j u_DG + (1 - omega_j) u_lim,
 *   omega_j = (max eta - eta_j) / (max eta - 1),
 * all other cells keep u_DG. */
int dgref_hybrid1d(const dgref_problem1d* P, double dt, const double* v, double* out,
                   int64_t* troubled)
{
    int rc = check1d(P);
    if (rc) return rc;
    const int K1 = P->k + 1;
    const int64_t n = P->n;
    const int nv = dgref_nvars(P->eq, 1);
    double* E = (double*)malloc(sizeof(double) * (size_t)n * (size_t)K1);
    double* eta = (double*)malloc(sizeof(double) * (size_t)n);
    if (!E || !eta) { free(E); free(eta); return DGREF_ERR_ARG; }
    rc = dgref_exponents1d(P, dt, v, E, eta);
    if (!rc) {
        double M = 0.0;
        for (int64_t j = 0; j < n; ++j)
            if (!(eta[j] <= M)) M = eta[j];
        int64_t cnt = 0;
        for (int64_t j = 0; j < n; ++j) {
            int hit = eta[j] > 1.0;
            double w = hit ? (M - eta[j]) / (M - 1.0) : 1.0;
            cnt += hit;
            for (int s = 0; s < nv; ++s)
                for (int l = 0; l < K1; ++l) {
                    double dg = U1(v, s, l, j);
                    if (hit && l > 0) {
                        /* mode 0: u_lim^0 = u_DG^0 (sigma^0 = 0), so the blend
                         * of two equal values is that value */
                        double lim = exp(-E[(size_t)j * K1 + l]) * dg;
                        U1(out, s, l, j) = w * dg + (1.0 - w) * lim;
                    } else {
                        U1(out, s, l, j) = dg;
                    }
                }
        }
        if (troubled) *troubled += cnt;
    }
    free(E);
    free(eta);
    return rc;
}

/* Post-stage operator applied after every RK stage (Sec. 3).
 * Reading of the damping duration: the split viscous problem is advanced
 * over the full step dt after every stage (filter_dt = 0); filter_dt = 1
 * uses the stage's own weight (1, 1/4, 2/3) of dt instead. */
/* ------------------------------------------------------------------------ */
/* Positivity-preserving limiter (Zhang and Shu; used after the filter in    */
/* the paper's Sec. 3.2 examples with extreme positivity demands)            */
/* ------------------------------------------------------------------------ */

/* Test points of a cell: the Gauss-Lobatto points with N = ceil((k+3)/2)
 * (they include both ends, where the fluxes are evaluated, and their rule
 * is exact for degree k, so the cell average is a convex combination of
 * the point values) and the Gauss points of the volume quadrature.
 * Gauss-Lobatto nodes: +-1 and the roots of P_{N-1}' (0 for N = 3,
 * +-sqrt(1/5) for N = 4).  V[i][l] = P_l at point i, taken from the same
 * tables the DG operator evaluates its traces and quadrature values with,
 * so a point value here is bitwise the value the fluxes will see. */
static int pp_points(const dgref_problem1d* P, double V[16][MAXK + 1])
{
    dgref_basis B;
    if (dgref_make_basis(P->k, P->nq, &B)) return 0;
    const int K1 = P->k + 1;
    const int N = (P->k + 4) / 2 < 2 ? 2 : (P->k + 4) / 2;
    int cnt = 0;
    for (int side = 0; side < 2; ++side, ++cnt)
        for (int l = 0; l < K1; ++l) V[cnt][l] = B.tr[side][l][0];
    if (N == 3) {
        for (int l = 0; l < K1; ++l) V[cnt][l] = dgref_legendre_deriv(l, 0, 0.0);
        ++cnt;
    }
    if (N == 4)
        for (int sgn = -1; sgn <= 1; sgn += 2, ++cnt)
            for (int l = 0; l < K1; ++l)
                V[cnt][l] = (double)legendre_deriv_ld(l, 0, (long double)sgn * sqrtl(0.2L));
    for (int q = 0; q < B.nq; ++q, ++cnt)
        for (int l = 0; l < K1; ++l) V[cnt][l] = B.phi[q][l];
    return cnt;
}

static void point_state1d(const dgref_problem1d* P, const double* u, int64_t j,
                          const double* Vi, double* w)
{
    const int K1 = P->k + 1;
    const int64_t n = P->n;
    for (int v = 0; v < 3; ++v) {
        double s = 0.0;
        for (int l = 0; l < K1; ++l) s += U1(u, v, l, j) * Vi[l];
        w[v] = s;
    }
}

static double pressure_of(double gamma, const double* w)
{
    return (gamma - 1.0) * (w[2] - 0.5 * w[1] * w[1] / w[0]);
}

/* The pressure as the flux and the wave speed evaluate it. */
static double pressure_flux(double gamma, const double* w)
{
    const double vel = w[1] / w[0];
    return (gamma - 1.0) * (w[2] - 0.5 * w[1] * vel);
}

/* Point value w and the sums wa of the magnitudes of its terms. */
static void point_state_abs1d(const dgref_problem1d* P, const double* u, int64_t j,
                              const double* Vi, double* w, double* wa)
{
    const int K1 = P->k + 1;
    const int64_t n = P->n;
    for (int v = 0; v < 3; ++v) {
        double s = 0.0, sa = 0.0;
        for (int l = 0; l < K1; ++l) {
            s += U1(u, v, l, j) * Vi[l];
            sa += fabs(U1(u, v, l, j) * Vi[l]);
        }
        w[v] = s;
        wa[v] = sa;
    }
}

/* Rounding margin of the pressure at a point (8 units of roundoff times
 * the magnitudes that cancel in E - m^2 / (2 rho)): near vacuum the point
 * pressure is the small difference of two large numbers, so a value below
 * this margin has no reliable sign. */
static double pp_margin(const double* w, const double* wa)
{
    const double ur = 0x1p-52;
    const double kin = 0.5 * w[1] * w[1] / w[0];
    return 8.0 * ur * (wa[2] + fabs(w[1]) * wa[1] / w[0] + kin * wa[0] / w[0]);
}

/* Limit cell j of u in place: scale the density's higher modes so the
 * density at every test point is >= eps_r, then all higher modes so the
 * pressure at each point is >= eps_p (for each point the largest t in
 * [0,1] with p(u_bar + t (u(x) - u_bar)) >= eps_p, found by bisection; p is
 * concave along that segment).  eps = min(1e-13, rho_bar, p(u_bar)) as in
 * Zhang and Shu; here eps_r = max(eps, 8 u sum_l |rho_l P_l|) and eps_p =
 * max(eps, the rounding margin of the point's pressure), which equal eps
 * in exact arithmetic.  Cell averages are not changed.  The scaled cell is
 * then checked point by point in the arithmetic of the fluxes, its higher
 * modes halved until density and pressure are positive there (dropped after
 * 50 halvings; with the margins this does not occur in practice). */
static void pp_limit_cell(const dgref_problem1d* P, double* u, int64_t j)
{
    const int K1 = P->k + 1;
    const int64_t n = P->n;
    double ub[3];
    for (int v = 0; v < 3; ++v) ub[v] = U1(u, v, 0, j);
    double pb = pressure_of(P->gamma, ub);
    if (!(ub[0] > 0.0) || !(pb > 0.0)) return; /* inadmissible average: not limitable */
    double eps = 1e-13;
    if (ub[0] < eps) eps = ub[0];
    if (pb < eps) eps = pb;
    double V[16][MAXK + 1];
    int np = pp_points(P, V);
    /* density */
    double rmin = INFINITY, eps_r = eps;
    for (int i = 0; i < np; ++i) {
        double w[3], wa[3];
        point_state_abs1d(P, u, j, V[i], w, wa);
        if (w[0] < rmin) rmin = w[0];
        double m = 8.0 * 0x1p-52 * wa[0];
        if (m > eps_r) eps_r = m;
    }
    if (eps_r > ub[0]) eps_r = ub[0];
    if (rmin < eps_r) {
        double th = (ub[0] - eps_r) / (ub[0] - rmin);
        if (th < 0.0) th = 0.0;
        for (int l = 1; l < K1; ++l) U1(u, 0, l, j) *= th;
    }
    /* pressure */
    double theta = 1.0;
    for (int i = 0; i < np; ++i) {
        double w[3], wa[3];
        point_state_abs1d(P, u, j, V[i], w, wa);
        double eps_p = eps;
        if (w[0] > 0.0) {
            double m = pp_margin(w, wa);
            if (m > eps_p) eps_p = m;
        }
        if (eps_p > pb) eps_p = pb;
        if (pressure_of(P->gamma, w) >= eps_p) continue;
        double lo = 0.0, hi = 1.0;
        for (int it = 0; it < 60; ++it) {
            double mid = 0.5 * (lo + hi), wm[3];
            for (int v = 0; v < 3; ++v) wm[v] = ub[v] + mid * (w[v] - ub[v]);
            if (pressure_of(P->gamma, wm) >= eps_p)
                lo = mid;
            else
                hi = mid;
        }
        if (lo < theta) theta = lo;
    }
    if (theta < 1.0)
        for (int v = 0; v < 3; ++v)
            for (int l = 1; l < K1; ++l) U1(u, v, l, j) *= theta;
    /* positivity in the fluxes' own arithmetic */
    for (int halving = 0; halving <= 50; ++halving) {
        int ok = 1;
        for (int i = 0; i < np && ok; ++i) {
            double w[3];
            point_state1d(P, u, j, V[i], w);
            ok = w[0] > 0.0 && pressure_flux(P->gamma, w) > 0.0;
        }
        if (ok) return;
        const double f = halving < 50 ? 0.5 : 0.0;
        for (int v = 0; v < 3; ++v)
            for (int l = 1; l < K1; ++l) U1(u, v, l, j) *= f;
    }
}

int dgref_pp_limit1d(const dgref_problem1d* P, double* u)
{
    int rc = check1d(P);
    if (rc) return rc;
    if (P->eq != DGREF_EULER) return DGREF_OK;
#pragma omp parallel for schedule(static) if (P->n >= 4096)
    for (int64_t j = 0; j < P->n; ++j) pp_limit_cell(P, u, j);
    return DGREF_OK;
}

int dgref_post1d(const dgref_problem1d* P, int stage, double dt, const double* v,
                 double* out, int64_t* troubled)
{
    static const double stage_weight[3] = {1.0, 0.25, 2.0 / 3.0};
    int rc = check1d(P);
    if (rc) return rc;
    double tau = (P->filter_dt == 1) ? dt * stage_weight[stage] : dt;
    const size_t ndof = (size_t)dgref_nvars(P->eq, 1) * (size_t)(P->k + 1) * (size_t)P->n;
    if (P->filter == DGREF_FILTER_JUMP)
        rc = dgref_filter1d(P, tau, v, out);
    else if (P->filter == DGREF_FILTER_HYBRID)
        rc = dgref_hybrid1d(P, tau, v, out, troubled);
    else if (out != v)
        memcpy(out, v, sizeof(double) * ndof);
    if (!rc && P->pp) rc = dgref_pp_limit1d(P, out);
    return rc;
}

/* One SSP-RK3 step with the post-stage operator after each stage (err_rk1,
 * err_rk2).  bflux (nullable) accumulates dt * sum_s b_s (fhat_right -
 * fhat_left) with the effective weights b = (1/6, 1/6, 2/3). */
static int averages_admissible(const dgref_problem1d* P, const double* u)
{
    const int K1 = P->k + 1;
    const int64_t n = P->n;
    for (int64_t j = 0; j < n; ++j) {
        double w[3] = {U1(u, 0, 0, j), U1(u, 1, 0, j), U1(u, 2, 0, j)};
        if (!(w[0] > 0.0) || !(pressure_of(P->gamma, w) > 0.0)) return 0;
    }
    return 1;
}

/* One SSP-RK3 step with the post-stage operator after every stage.  With
 * the positivity limiter, a stage whose cell averages leave the admissible
 * set (the CFL bound of the positivity argument failed for the stage
 * states) rejects the step: DGREF_ERR_POSITIVITY is returned and u, bflux
 * and troubled are left untouched, so the caller can retry with a smaller
 * dt. */
int dgref_step1d(const dgref_problem1d* P, double dt, double* u, double* bflux,
                 int64_t* troubled)
{
    static const double b[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
    int rc = check1d(P);
    if (rc) return rc;
    const int nv = dgref_nvars(P->eq, 1);
    const int64_t n = P->n;
    const size_t ndof = (size_t)nv * (size_t)(P->k + 1) * (size_t)n;
    double bf0[MAXV] = {0.0, 0.0, 0.0, 0.0};
    int64_t tr0 = troubled ? *troubled : 0;
    if (bflux)
        for (int v = 0; v < nv; ++v) bf0[v] = bflux[v];
    double* un = (double*)malloc(sizeof(double) * ndof);
    double* us = (double*)malloc(sizeof(double) * ndof);
    double* w = (double*)malloc(sizeof(double) * ndof);
    double* fh = (double*)malloc(sizeof(double) * (size_t)nv * (size_t)(n + 1));
    if (!un || !us || !w || !fh) { rc = DGREF_ERR_ARG; goto done; }
    memcpy(un, u, sizeof(double) * ndof);
    memcpy(us, u, sizeof(double) * ndof);
    for (int s = 0; s < 3 && !rc; ++s) {
        rc = dgref_stage1d(P, s, dt, un, us, w, fh);
        if (rc) break;
        if (bflux)
            for (int v = 0; v < nv; ++v)
                bflux[v] += dt * b[s] *
                            (fh[(size_t)v * (size_t)(n + 1) + (size_t)n] - fh[(size_t)v * (size_t)(n + 1)]);
        rc = dgref_post1d(P, s, dt, w, us, troubled);
        if (!rc && P->pp && P->eq == DGREF_EULER && !averages_admissible(P, us))
            rc = DGREF_ERR_POSITIVITY;
    }
    if (!rc) {
        memcpy(u, us, sizeof(double) * ndof);
    } else {
        if (bflux)
            for (int v = 0; v < nv; ++v) bflux[v] = bf0[v];
        if (troubled) *troubled = tr0;
    }
done:
    free(un);
    free(us);
    free(w);
    free(fh);
    return rc;
}

/* Positivity of density and pressure at every quadrature and trace point
 * (Euler), and finiteness of every coefficient. */
int dgref_check1d(const dgref_problem1d* P, const double* u, double* min_rho, double* min_p,
                  int64_t* first_bad)
{
    int rc = check1d(P);
    if (rc) return rc;
    dgref_basis B;
    if ((rc = dgref_make_basis(P->k, P->nq, &B))) return rc;
    const int K1 = P->k + 1;
    const int64_t n = P->n;
    const int nv = dgref_nvars(P->eq, 1);
    double mr = INFINITY, mp = INFINITY;
    int status = DGREF_OK;
    int64_t bad = -1;
    for (int64_t j = 0; j < n; ++j) {
        int finite = 1;
        for (int s = 0; s < nv; ++s)
            for (int l = 0; l < K1; ++l)
                if (!isfinite(U1(u, s, l, j))) finite = 0;
        if (!finite) {
            if (status == DGREF_OK) { status = DGREF_ERR_NONFINITE; bad = j; }
            continue;
        }
        if (P->eq != DGREF_EULER) continue;
        for (int q = 0; q < B.nq + 2; ++q) {
            double uq[MAXV];
            for (int s = 0; s < nv; ++s) {
                double acc = 0.0;
                for (int l = 0; l < K1; ++l) {
                    double ph = (q < B.nq) ? B.phi[q][l] : B.tr[q - B.nq][l][0];
                    acc += U1(u, s, l, j) * ph;
                }
                uq[s] = acc;
            }
            double p = (P->gamma - 1.0) * (uq[2] - 0.5 * uq[1] * uq[1] / uq[0]);
            if (uq[0] < mr) mr = uq[0];
            if (p < mp) mp = p;
            if ((!(uq[0] > 0.0) || !(p > 0.0)) && status == DGREF_OK && !P->pp) {
                status = DGREF_ERR_POSITIVITY;
                bad = j;
            }
        }
        /* with the positivity limiter, point values sit at its margin eps
         * up to rounding: only an inadmissible cell average is an error */
        if (P->pp && status == DGREF_OK) {
            double w[3] = {U1(u, 0, 0, j), U1(u, 1, 0, j), U1(u, 2, 0, j)};
            double pb = (P->gamma - 1.0) * (w[2] - 0.5 * w[1] * w[1] / w[0]);
            if (!(w[0] > 0.0) || !(pb > 0.0)) {
                status = DGREF_ERR_POSITIVITY;
                bad = j;
            }
        }
    }
    if (min_rho) *min_rho = mr;
    if (min_p) *min_p = mp;
    if (first_bad) *first_bad = bad;
    return status;
}

/* Time loop: alpha from the cell averages, dt = cfl*h/alpha, the last step
 * clamped to end exactly at t_end. */
int dgref_run1d(const dgref_problem1d* P, double t_end, int64_t max_steps, double* u,
                dgref_report* rep)
{
    int rc = check1d(P);
    if (rc) return rc;
    const int K1 = P->k + 1;
    const int64_t n = P->n;
    const int nv = dgref_nvars(P->eq, 1);
    const double h = (P->hi - P->lo) / (double)n;
    dgref_report r;
    memset(&r, 0, sizeof r);
    r.dt_min = INFINITY;
    r.first_bad_cell = -1;
    double t = 0.0;
    while (t < t_end && r.steps < max_steps) {
        double alpha = dgref_max_wavespeed1d(P, u);
        if (!isfinite(alpha)) { rc = DGREF_ERR_NONFINITE; break; }
        double dt = P->cfl * h / alpha;
        /* a time step too small to advance t ends the run */
        if (!(t + dt > t)) { rc = DGREF_ERR_NONFINITE; break; }
        int last = 0;
        if (t + dt >= t_end) { dt = t_end - t; last = 1; }
        rc = dgref_step1d(P, dt, u, r.boundary_flux, &r.troubled_cells);
        /* positivity limiter: a rejected step is retried with half the time
         * step (Zhang and Shu's remedy when a stage violates the CFL bound
         * of the positivity argument) */
        for (int tries = 0; rc == DGREF_ERR_POSITIVITY && P->pp && tries < DGREF_MAX_RETRIES;
             ++tries) {
            dt *= 0.5;
            last = 0;
            r.restarts++;
            rc = dgref_step1d(P, dt, u, r.boundary_flux, &r.troubled_cells);
        }
        if (rc) break;
        t = last ? t_end : t + dt;
        r.steps++;
        if (dt < r.dt_min) r.dt_min = dt;
        if (dt > r.dt_max) r.dt_max = dt;
    }
    r.t = t;
    for (int s = 0; s < nv; ++s) {
        double q = 0.0;
        for (int64_t j = 0; j < n; ++j) q += h * U1(u, s, 0, j);
        r.ledger[s] = q;
    }
    int crc = dgref_check1d(P, u, &r.min_rho, &r.min_p, &r.first_bad_cell);
    if (!rc) rc = crc;
    r.status = rc;
    if (rep) *rep = r;
    (void)K1;
    return rc;
}
