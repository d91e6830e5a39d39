/*
 * dgref.h — FP64 CPU oracle for the RKDG scheme with the jump filter
 * (Wei, Zhou, Xia, "The jump filter in the discontinuous Galerkin method
 * for hyperbolic conservation laws", arXiv:2407.19169).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no source,
 * header, table or constant generator with the GPU library.
 *
 * State layout (the same layout the inputs are exchanged in):
 *   1D: u[(var * (k+1) + l) * n + j]            modal coefficient u_j^{l,(var)}
 *   2D: u[((var * nm + p*(k+1) + q) * ny + jy) * nx + ix]   Q^k tensor modes
 * with the standard Legendre basis P_l(xi), P_0 = 1, so mode 0 is the cell
 * average (Sec. 2.1, basis expansion (eq:GLbasisequation)).
 */
#ifndef DGREF_H
#define DGREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { DGREF_ADVECTION = 0, DGREF_BURGERS = 1, DGREF_EULER = 2 };
enum { DGREF_PERIODIC = 0, DGREF_OUTFLOW = 1, DGREF_REFLECT = 2, DGREF_DIRICHLET = 3 };
enum { DGREF_FILTER_NONE = 0, DGREF_FILTER_JUMP = 1, DGREF_FILTER_HYBRID = 2 };
/* Interface fluxes: local Lax-Friedrichs (the paper's computations), and
 * HLL / HLLC (named in Sec. 3 as alternatives; Euler only). */
enum { DGREF_FLUX_LLF = 0, DGREF_FLUX_HLL = 1, DGREF_FLUX_HLLC = 2 };

/* Status bits of a run. */
enum { DGREF_OK = 0, DGREF_ERR_ARG = -1, DGREF_ERR_NONFINITE = -4, DGREF_ERR_POSITIVITY = -5 };

typedef struct {
    int eq;              /* DGREF_ADVECTION / BURGERS / EULER                  */
    int k;               /* polynomial degree, 0..4                            */
    int nq;              /* Gauss points per direction (0 -> k+1)              */
    int filter;          /* DGREF_FILTER_*                                     */
    int filter_dt;       /* 0: damping time = full dt after every stage;
                            1: damping time = dt times the stage's RK weight   */
    int bc[2];           /* left, right boundary                               */
    int64_t n;           /* cells                                              */
    double lo, hi;       /* domain                                             */
    double gamma;        /* ratio of specific heats (Euler)                    */
    double adv_speed;    /* a in f(u) = a u (advection)                        */
    double cfl;          /* dt = cfl * h / alpha                               */
    double dirichlet[2][3]; /* prescribed boundary states (conserved vars)     */
    int pp;              /* 1: positivity-preserving limiter after the filter   */
    int flux;            /* DGREF_FLUX_*: interface flux (HLL / HLLC: Euler)    */
} dgref_problem1d;

typedef struct {
    int eq, k, nq, filter, filter_dt;
    int bc[4];           /* x-lo, x-hi, y-lo, y-hi                             */
    int64_t nx, ny;
    double xlo, xhi, ylo, yhi;
    double gamma;
    double adv_speed[2];
    double cfl;
    double dirichlet[4][4];
    /* double-Mach-reflection boundaries: the shock line is
     * x = shock_x0 + y / sqrt(3) + shock_speed * t; post/pre are the
     * conserved states behind (left of) and ahead of it */
    double shock_x0, shock_speed;
    double post[4], pre[4];
    int cf_reading; /* mesh factors (m_x, m_y) of the Euler coefficient
                       (c_fx, c_fy) = (m_x beta^x, m_y beta^y) / (4 lambda_pq H-bar):
                       0: (h_x, h_y), as printed in Sec. 2.4 (default);
                       1: (h_y, h_x), as printed in Sec. 3.2;
                       2: (1, 1), without mesh factors */
    int basis;     /* 0: Q^k tensor product; 1: P^k total degree (p + q <= k) */
    int flux;      /* DGREF_FLUX_*: interface flux (HLL / HLLC: Euler) */
    int pp;        /* 1: positivity-preserving limiter after the filter (Euler) */
} dgref_problem2d;

typedef struct {
    int64_t steps;
    double t, dt_min, dt_max;
    double ledger[4];          /* sum_j |K_j| * cell average, per variable     */
    double boundary_flux[4];   /* time integral of the net outward flux        */
    int64_t troubled_cells;    /* hybrid: troubled cells summed over stages    */
    double min_rho, min_p;     /* Euler: over trace and quadrature points      */
    double max_exponent;       /* largest damping exponent applied             */
    int status;
    int64_t first_bad_cell;
    int64_t restarts;          /* steps retried with half dt (positivity limiter) */
} dgref_report;

/* retries of one step with halved dt before the run stops */
#define DGREF_MAX_RETRIES 40

int dgref_nvars(int eq, int dim);
int dgref_num_threads(void);   /* OpenMP threads the cell loops use */
void dgref_set_threads(int n); /* set them (n > 0) */

/* ---- basis tables (exposed so tests can pin them) ---- */
int dgref_gauss(int q, double* x, double* w);
/* value of d^m/dxi^m P_l at xi */
double dgref_legendre_deriv(int l, int m, double xi);
/* nodes, weights, P_l and P_l' at the nodes of the rule of nq (0: k+1) points */
int dgref_basis_tables(int k, int nq, double* x, double* w, double* phi, double* dphi);

/* ---- 1D ---- */
int dgref_residual1d(const dgref_problem1d* P, const double* u, double* L, double* fhat);
double dgref_max_wavespeed1d(const dgref_problem1d* P, const double* u);
int dgref_stage1d(const dgref_problem1d* P, int stage, double dt, const double* un,
                  const double* us, double* out, double* fhat);
int dgref_exponents1d(const dgref_problem1d* P, double dt, const double* v, double* E,
                      double* eta);
int dgref_filter1d(const dgref_problem1d* P, double dt, const double* v, double* out);
int dgref_hybrid1d(const dgref_problem1d* P, double dt, const double* v, double* out,
                   int64_t* troubled);
int dgref_post1d(const dgref_problem1d* P, int stage, double dt, const double* v,
                 double* out, int64_t* troubled);
int dgref_pp_limit1d(const dgref_problem1d* P, double* u);
/* The interface flux of P between the states ul (left) and ur (right);
 * 2D: across a face of normal +x (dir 0) or +y (dir 1). */
int dgref_numflux1d(const dgref_problem1d* P, const double* ul, const double* ur, double* fh);
int dgref_numflux2d(const dgref_problem2d* P, int dir, const double* ul, const double* ur,
                    double* fh);
int dgref_step1d(const dgref_problem1d* P, double dt, double* u, double* bflux,
                 int64_t* troubled);
int dgref_run1d(const dgref_problem1d* P, double t_end, int64_t max_steps, double* u,
                dgref_report* rep);
int dgref_check1d(const dgref_problem1d* P, const double* u, double* min_rho,
                  double* min_p, int64_t* first_bad);

/* ---- 2D, Q^k tensor-product Legendre ---- */
int dgref_residual2d(const dgref_problem2d* P, double t, const double* u, double* L);
double dgref_max_wavespeed2d(const dgref_problem2d* P, const double* u);
int dgref_stage2d(const dgref_problem2d* P, int stage, double t, double dt, const double* un,
                  const double* us, double* out);
int dgref_exponents2d(const dgref_problem2d* P, double t, double dt, const double* v, double* E,
                      double* eta);
int dgref_post2d(const dgref_problem2d* P, int stage, double t, double dt, const double* v,
                 double* out, int64_t* troubled);
int dgref_check2d(const dgref_problem2d* P, const double* u, double* min_rho, double* min_p,
                  int64_t* first_bad);
int dgref_pp_limit2d(const dgref_problem2d* P, double* u);
/* Reference-coordinate test points of the 2D positivity limiter: xi[i],
 * eta[i] for i < return value (at most 6 nq + nq^2). */
int dgref_pp_points2d(const dgref_problem2d* P, double* xi, double* eta);
int dgref_step2d(const dgref_problem2d* P, double t, double dt, double* u, int64_t* troubled);
int dgref_run2d(const dgref_problem2d* P, double t_end, int64_t max_steps, double* u,
                dgref_report* rep);

#ifdef __cplusplus
}
#endif
#endif
