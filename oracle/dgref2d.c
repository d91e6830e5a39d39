/*
 * dgref2d.c — 2D part of the FP64 CPU oracle (arXiv:2407.19169, Sec. 2.3
 * two-dimensional scheme and filter, Sec. 2.4 systems, Sec. 3.2 Euler).
 * TEST INFRASTRUCTURE ONLY; shares nothing with the GPU library.
 *
 * Space: tensor-product Legendre Q^k on a uniform Cartesian mesh, mode
 * (p, q) = P_p(xi) P_q(eta) with p the x-degree, stored at index p*(k+1)+q.
 * Every quantity is computed per cell with plain loops; interface values
 * are recomputed from the two neighbouring cells wherever they are needed.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "dgref.h"
#include "dgref_internal.h"

#define NMAX ((MAXK + 1) * (MAXK + 1))
/* test points of the positivity limiter: 2 x (3 Lobatto x nq) + nq x nq */
#define PPMAX (6 * MAXQ + MAXQ * MAXQ)

typedef struct {
    const dgref_problem2d* P;
    dgref_basis B;
    int k, K1, NM, nv;
    int64_t nx, ny;
    double hx, hy;
} ctx2d;

static int check2d(const dgref_problem2d* P)
{
    if (!P || P->nx < 1 || P->ny < 1 || P->k < 0 || P->k > 3) return DGREF_ERR_ARG;
    if (P->eq != DGREF_ADVECTION && P->eq != DGREF_EULER) return DGREF_ERR_ARG;
    if (!(P->xhi > P->xlo) || !(P->yhi > P->ylo)) return DGREF_ERR_ARG;
    for (int s = 0; s < 4; ++s) {
        if (P->bc[s] < 0 || P->bc[s] > 5) return DGREF_ERR_ARG;
        if (P->eq != DGREF_EULER && (P->bc[s] == DGREF_REFLECT || P->bc[s] >= 4)) return DGREF_ERR_ARG;
    }
    if ((P->bc[0] == DGREF_PERIODIC) != (P->bc[1] == DGREF_PERIODIC)) return DGREF_ERR_ARG;
    if ((P->bc[2] == DGREF_PERIODIC) != (P->bc[3] == DGREF_PERIODIC)) return DGREF_ERR_ARG;
    if (P->cf_reading < 0 || P->cf_reading > 2) return DGREF_ERR_ARG;
    if (P->pp && P->eq != DGREF_EULER) return DGREF_ERR_ARG;
    return DGREF_OK;
}

static int make_ctx(const dgref_problem2d* P, ctx2d* C)
{
    int rc = check2d(P);
    if (rc) return rc;
    C->P = P;
    if ((rc = dgref_make_basis(P->k, P->nq, &C->B))) return rc;
    C->k = P->k;
    C->K1 = P->k + 1;
    C->NM = C->K1 * C->K1;
    C->nv = dgref_nvars(P->eq, 2);
    C->nx = P->nx;
    C->ny = P->ny;
    C->hx = (P->xhi - P->xlo) / (double)P->nx;
    C->hy = (P->yhi - P->ylo) / (double)P->ny;
    return DGREF_OK;
}

static inline double U(const ctx2d* C, const double* u, int v, int m, int64_t ix, int64_t jy)
{
    return u[(((size_t)v * C->NM + m) * C->ny + jy) * C->nx + ix];
}
static inline double* Up(const ctx2d* C, double* u, int v, int m, int64_t ix, int64_t jy)
{
    return &u[(((size_t)v * C->NM + m) * C->ny + jy) * C->nx + ix];
}

/* ------------------------------------------------------------- physics -- */
/* Normal flux in direction dir (0: x, 1: y) (Sec. 3.2 Euler flux). */
static void flux2d(const dgref_problem2d* P, int dir, const double* u, double* f)
{
    if (P->eq == DGREF_ADVECTION) {
        f[0] = P->adv_speed[dir] * u[0];
        return;
    }
    double rho = u[0], mx = u[1], my = u[2], E = u[3];
    double vx = mx / rho, vy = my / rho;
    double p = (P->gamma - 1.0) * (E - 0.5 * (mx * vx + my * vy));
    double vn = dir == 0 ? vx : vy;
    f[0] = rho * vn;
    f[1] = mx * vn + (dir == 0 ? p : 0.0);
    f[2] = my * vn + (dir == 1 ? p : 0.0);
    f[3] = vn * (E + p);
}

static double pressure2d(const dgref_problem2d* P, const double* u)
{
    return (P->gamma - 1.0) * (u[3] - 0.5 * (u[1] * u[1] + u[2] * u[2]) / u[0]);
}

/* Largest wave speed along dir: |u_n| + c (Euler), |a_n| (advection). */
static double lambda2d(const dgref_problem2d* P, int dir, const double* u)
{
    if (P->eq == DGREF_ADVECTION) return fabs(P->adv_speed[dir]);
    double p = pressure2d(P, u);
    return fabs(u[1 + dir] / u[0]) + sqrt(P->gamma * p / u[0]);
}

static double enthalpy2d(const dgref_problem2d* P, const double* u)
{
    if (P->eq != DGREF_EULER) return 1.0;
    return (u[3] + pressure2d(P, u)) / u[0];
}

/* LLF flux across a face with normal +dir. */
static void llf2d(const dgref_problem2d* P, int dir, const double* ul, const double* ur, double* fh)
{
    int nv = dgref_nvars(P->eq, 2);
    double fl[MAXV], fr[MAXV];
    flux2d(P, dir, ul, fl);
    flux2d(P, dir, ur, fr);
    double al = lambda2d(P, dir, ul), ar = lambda2d(P, dir, ur);
    double a = al > ar ? al : ar;
    for (int v = 0; v < nv; ++v) fh[v] = 0.5 * (fl[v] + fr[v]) - 0.5 * a * (ur[v] - ul[v]);
}

/* The interface flux the problem asks for: LLF, or HLL / HLLC (Euler). */
static void numflux2d(const dgref_problem2d* P, int dir, const double* ul, const double* ur,
                      double* fh)
{
    if (P->eq == DGREF_EULER && P->flux != DGREF_FLUX_LLF)
        dgref_hll_flux(P->flux, 4, dir, P->gamma, ul, ur, fh);
    else
        llf2d(P, dir, ul, ur, fh);
}

int dgref_numflux2d(const dgref_problem2d* P, int dir, const double* ul, const double* ur,
                    double* fh)
{
    if (!P || P->flux < DGREF_FLUX_LLF || P->flux > DGREF_FLUX_HLLC || dir < 0 || dir > 1)
        return DGREF_ERR_ARG;
    numflux2d(P, dir, ul, ur, fh);
    return DGREF_OK;
}

/* --------------------------------------------------------- evaluation -- */
/* u at reference point given P_p(xi) values px[p] and P_q(eta) values py[q]. */
static void point_value(const ctx2d* C, const double* u, int64_t ix, int64_t jy, const double* px,
                        const double* py, double* out)
{
    for (int v = 0; v < C->nv; ++v) {
        double s = 0.0;
        for (int p = 0; p < C->K1; ++p)
            for (int q = 0; q < C->K1; ++q) s += U(C, u, v, p * C->K1 + q, ix, jy) * px[p] * py[q];
        out[v] = s;
    }
}

/* d^a1/dx^a1 d^a2/dy^a2 u at corner (sx, sy) (0: -1 side, 1: +1 side). */
static void corner_deriv(const ctx2d* C, const double* u, int64_t ix, int64_t jy, int a1, int a2,
                         int sx, int sy, double* out)
{
    double scale = pow(2.0 / C->hx, a1) * pow(2.0 / C->hy, a2);
    for (int v = 0; v < C->nv; ++v) {
        double s = 0.0;
        for (int p = 0; p < C->K1; ++p)
            for (int q = 0; q < C->K1; ++q)
                s += U(C, u, v, p * C->K1 + q, ix, jy) * C->B.tr[sx][p][a1] * C->B.tr[sy][q][a2];
        out[v] = scale * s;
    }
}

/* Position of the shock line of the double-Mach-reflection problem. */
static double shock_x(const dgref_problem2d* P, double y, double t)
{
    return P->shock_x0 + y / sqrt(3.0) + P->shock_speed * t;
}

/* Ghost state outside boundary side (0 x-lo, 1 x-hi, 2 y-lo, 3 y-hi) at the
 * physical point (x, y), time t, from the interior trace (for the flux).
 * Reading of the boundary treatment: outflow copies, reflection negates
 * the normal momentum, Dirichlet (inflow) imposes the given state; the
 * double-Mach wall imposes the post-shock state for x < shock_x0 and
 * reflects beyond; the double-Mach top imposes the exact moving shock. */
static void ghost2d(const dgref_problem2d* P, int side, double x, double y, double t,
                    const double* in, double* g)
{
    int nv = dgref_nvars(P->eq, 2);
    int bc = P->bc[side];
    int dir = side / 2;
    if (bc == DGREF_DIRICHLET) {
        for (int v = 0; v < nv; ++v) g[v] = P->dirichlet[side][v];
        return;
    }
    if (bc == 4 /* DMR wall */) {
        if (x < P->shock_x0) {
            for (int v = 0; v < nv; ++v) g[v] = P->post[v];
            return;
        }
        bc = DGREF_REFLECT;
    }
    if (bc == 5 /* DMR top */) {
        const double* st = x < shock_x(P, y, t) ? P->post : P->pre;
        for (int v = 0; v < nv; ++v) g[v] = st[v];
        return;
    }
    for (int v = 0; v < nv; ++v) g[v] = in[v];
    if (bc == DGREF_REFLECT) g[1 + dir] = -in[1 + dir];
}

/* |ghost - inner| of the mixed derivative (a1, a2) at a boundary corner,
 * from the interior one-sided value (jump filter at physical boundaries).
 * Outflow: zero jump; reflection: the ghost is the mirror image, so the
 * derivative picks up (-1)^(normal order) and the normal momentum a sign;
 * prescribed states have zero derivatives. */
static void ghost_jump2d(const dgref_problem2d* P, int side, double x, double y, double t, int a1,
                         int a2, const double* in, double* jmp)
{
    int nv = dgref_nvars(P->eq, 2);
    int bc = P->bc[side];
    int dir = side / 2;
    const double* st = NULL;
    if (bc == DGREF_DIRICHLET) st = P->dirichlet[side];
    if (bc == 4) {
        if (x < P->shock_x0)
            st = P->post;
        else
            bc = DGREF_REFLECT;
    }
    if (bc == 5) st = x < shock_x(P, y, t) ? P->post : P->pre;
    for (int v = 0; v < nv; ++v) {
        if (st) {
            jmp[v] = (a1 == 0 && a2 == 0) ? fabs(st[v] - in[v]) : fabs(in[v]);
        } else if (bc == DGREF_REFLECT) {
            int an = dir == 0 ? a1 : a2;
            double sgn = (an % 2) ? -1.0 : 1.0;
            if (v == 1 + dir) sgn = -sgn;
            jmp[v] = fabs(sgn * in[v] - in[v]);
        } else {
            jmp[v] = 0.0;
        }
    }
}

/* neighbour index along an axis with periodic wrap; -1 if outside */
static int64_t nbr(int64_t i, int64_t n, int periodic)
{
    if (i >= 0 && i < n) return i;
    if (!periodic) return -1;
    return (i % n + n) % n;
}

/* --------------------------------------------------------- residual -- */
/* Interface flux through the x-face at the left (side 0) or right (side 1) of
 * cell (ix, jy) at the edge Gauss point b. */
static void xface_flux(const ctx2d* C, double t, const double* u, int64_t ix, int64_t jy, int side,
                       int b, double* fh)
{
    const dgref_problem2d* P = C->P;
    double py[MAXK + 1], pin[MAXK + 1], pout[MAXK + 1];
    for (int q = 0; q < C->K1; ++q) py[q] = C->B.phi[b][q];
    for (int p = 0; p < C->K1; ++p) {
        pin[p] = C->B.tr[side][p][0];      /* own cell at xi = -1 / +1 */
        pout[p] = C->B.tr[1 - side][p][0]; /* neighbour at the other end */
    }
    double uin[MAXV], uout[MAXV];
    point_value(C, u, ix, jy, pin, py, uin);
    int64_t jx = nbr(ix + (side ? 1 : -1), C->nx, P->bc[0] == DGREF_PERIODIC);
    double x = P->xlo + (side ? ix + 1 : ix) * C->hx;
    double y = P->ylo + (jy + 0.5) * C->hy + 0.5 * C->hy * C->B.xq[b];
    if (jx >= 0)
        point_value(C, u, jx, jy, pout, py, uout);
    else
        ghost2d(P, side, x, y, t, uin, uout);
    if (side)
        numflux2d(P, 0, uin, uout, fh);
    else
        numflux2d(P, 0, uout, uin, fh);
}

static void yface_flux(const ctx2d* C, double t, const double* u, int64_t ix, int64_t jy, int side,
                       int a, double* fh)
{
    const dgref_problem2d* P = C->P;
    double px[MAXK + 1], qin[MAXK + 1], qout[MAXK + 1];
    for (int p = 0; p < C->K1; ++p) px[p] = C->B.phi[a][p];
    for (int q = 0; q < C->K1; ++q) {
        qin[q] = C->B.tr[side][q][0];
        qout[q] = C->B.tr[1 - side][q][0];
    }
    double uin[MAXV], uout[MAXV];
    point_value(C, u, ix, jy, px, qin, uin);
    int64_t jj = nbr(jy + (side ? 1 : -1), C->ny, P->bc[2] == DGREF_PERIODIC);
    double x = P->xlo + (ix + 0.5) * C->hx + 0.5 * C->hx * C->B.xq[a];
    double y = P->ylo + (side ? jy + 1 : jy) * C->hy;
    if (jj >= 0)
        point_value(C, u, ix, jj, px, qout, uout);
    else
        ghost2d(P, 2 + side, x, y, t, uin, uout);
    if (side)
        numflux2d(P, 1, uin, uout, fh);
    else
        numflux2d(P, 1, uout, uin, fh);
}

/* Residual of one cell (Sec. 2.3 scheme without the viscous term, with
 * v = P_p(xi) P_q(eta)):
 *   hx hy / ((2p+1)(2q+1)) du^{pq}/dt =
 *       (hy/2) sum_ab w_a w_b F1 P_p'(xi_a) P_q(eta_b)
 *     + (hx/2) sum_ab w_a w_b F2 P_p(xi_a) P_q'(eta_b)
 *     - (hy/2) sum_b w_b [Fhat1(i+1/2) P_p(1) - Fhat1(i-1/2) P_p(-1)] P_q(eta_b)
 *     - (hx/2) sum_a w_a [Fhat2(j+1/2) P_q(1) - Fhat2(j-1/2) P_q(-1)] P_p(xi_a) */
static void cell_residual(const ctx2d* C, double t, const double* u, int64_t ix, int64_t jy,
                          double L[][NMAX])
{
    const dgref_problem2d* P = C->P;
    const int K1 = C->K1, nq = C->B.nq, nv = C->nv;
    double acc[MAXV][NMAX];
    memset(acc, 0, sizeof acc);
    for (int a = 0; a < nq; ++a)
        for (int b = 0; b < nq; ++b) {
            double px[MAXK + 1], py[MAXK + 1], uq[MAXV], f1[MAXV], f2[MAXV];
            for (int p = 0; p < K1; ++p) px[p] = C->B.phi[a][p];
            for (int q = 0; q < K1; ++q) py[q] = C->B.phi[b][q];
            point_value(C, u, ix, jy, px, py, uq);
            flux2d(P, 0, uq, f1);
            flux2d(P, 1, uq, f2);
            double w = C->B.wq[a] * C->B.wq[b];
            for (int v = 0; v < nv; ++v)
                for (int p = 0; p < K1; ++p)
                    for (int q = 0; q < K1; ++q)
                        acc[v][p * K1 + q] +=
                            0.5 * C->hy * w * f1[v] * C->B.dphi[a][p] * C->B.phi[b][q] +
                            0.5 * C->hx * w * f2[v] * C->B.phi[a][p] * C->B.dphi[b][q];
        }
    for (int b = 0; b < nq; ++b) {
        double fl[MAXV], fr[MAXV];
        xface_flux(C, t, u, ix, jy, 0, b, fl);
        xface_flux(C, t, u, ix, jy, 1, b, fr);
        for (int v = 0; v < nv; ++v)
            for (int p = 0; p < K1; ++p)
                for (int q = 0; q < K1; ++q)
                    acc[v][p * K1 + q] -= 0.5 * C->hy * C->B.wq[b] *
                                          (fr[v] * C->B.tr[1][p][0] - fl[v] * C->B.tr[0][p][0]) *
                                          C->B.phi[b][q];
    }
    for (int a = 0; a < nq; ++a) {
        double fb[MAXV], ft[MAXV];
        yface_flux(C, t, u, ix, jy, 0, a, fb);
        yface_flux(C, t, u, ix, jy, 1, a, ft);
        for (int v = 0; v < nv; ++v)
            for (int p = 0; p < K1; ++p)
                for (int q = 0; q < K1; ++q)
                    acc[v][p * K1 + q] -= 0.5 * C->hx * C->B.wq[a] *
                                          (ft[v] * C->B.tr[1][q][0] - fb[v] * C->B.tr[0][q][0]) *
                                          C->B.phi[a][p];
    }
    for (int v = 0; v < nv; ++v)
        for (int p = 0; p < K1; ++p)
            for (int q = 0; q < K1; ++q) {
                double mass = C->hx * C->hy / ((2.0 * p + 1.0) * (2.0 * q + 1.0));
                /* P^k (basis 1): the modes with p + q > k are not in the
                 * space and stay zero */
                L[v][p * K1 + q] = (P->basis == 1 && p + q > C->k) ? 0.0 : acc[v][p * K1 + q] / mass;
            }
}

int dgref_residual2d(const dgref_problem2d* P, double t, const double* u, double* L)
{
    ctx2d C;
    int rc = make_ctx(P, &C);
    if (rc) return rc;
#pragma omp parallel for schedule(static) if (C.nx * C.ny >= 4096)
    for (int64_t jy = 0; jy < C.ny; ++jy)
        for (int64_t ix = 0; ix < C.nx; ++ix) {
            double Lc[MAXV][NMAX];
            cell_residual(&C, t, u, ix, jy, Lc);
            for (int v = 0; v < C.nv; ++v)
                for (int m = 0; m < C.NM; ++m) *Up(&C, L, v, m, ix, jy) = Lc[v][m];
        }
    return DGREF_OK;
}

/* CFL: max over cells of lambda_x/hx + lambda_y/hy at the cell averages;
 * the step is dt = cfl / that. */
double dgref_max_wavespeed2d(const dgref_problem2d* P, const double* u)
{
    ctx2d C;
    if (make_ctx(P, &C)) return NAN;
    double amax = 0.0;
    for (int64_t jy = 0; jy < C.ny; ++jy)
        for (int64_t ix = 0; ix < C.nx; ++ix) {
            double ub[MAXV];
            for (int v = 0; v < C.nv; ++v) ub[v] = U(&C, u, v, 0, ix, jy);
            double a = lambda2d(P, 0, ub) / C.hx + lambda2d(P, 1, ub) / C.hy;
            if (!(a <= amax)) amax = a;
        }
    return amax;
}

/* SSP-RK3 stage (Shu-Osher form), unfiltered; t is the start of the step,
 * the residual of stage s is evaluated at t + (0, 1, 1/2)[s] dt. */
int dgref_stage2d(const dgref_problem2d* P, int stage, double t, double dt, const double* un,
                  const double* us, double* out)
{
    static const double ct[3] = {0.0, 1.0, 0.5};
    ctx2d C;
    int rc = make_ctx(P, &C);
    if (rc) return rc;
    if (stage < 0 || stage > 2) return DGREF_ERR_ARG;
    const double* src = stage == 0 ? un : us;
    const double ts = t + ct[stage] * dt;
#pragma omp parallel for schedule(static) if (C.nx * C.ny >= 4096)
    for (int64_t jy = 0; jy < C.ny; ++jy)
        for (int64_t ix = 0; ix < C.nx; ++ix) {
            double Lc[MAXV][NMAX];
            cell_residual(&C, ts, src, ix, jy, Lc);
            for (int v = 0; v < C.nv; ++v)
                for (int m = 0; m < C.NM; ++m) {
                    double adv = U(&C, src, v, m, ix, jy) + dt * Lc[v][m];
                    double unv = U(&C, un, v, m, ix, jy);
                    double o = stage == 0 ? adv : stage == 1 ? 0.75 * unv + 0.25 * adv
                                                             : unv / 3.0 + 2.0 * adv / 3.0;
                    *Up(&C, out, v, m, ix, jy) = o;
                }
        }
    return DGREF_OK;
}

/* ------------------------------------------------------------ filter -- */
/* Edge-averaged jumps (trapezoidal rule along each edge) of every mixed
 * derivative d^a of each variable, summed over the two vertical (Jx) and
 * the two horizontal (Jy) edges of cell (ix, jy):
 *   Jx[a1][a2][v] = 1/2 sum_{faces x_{i-1/2}, x_{i+1/2}} sum_{corners y_{j-1/2}, y_{j+1/2}} |[d^a u]|. */
static void cell_jumps(const ctx2d* C, double t, const double* u, int64_t ix, int64_t jy,
                       double Jx[][MAXK + 1][MAXV], double Jy[][MAXK + 1][MAXV])
{
    const dgref_problem2d* P = C->P;
    const int K1 = C->K1, nv = C->nv;
    for (int a1 = 0; a1 < K1; ++a1)
        for (int a2 = 0; a2 < K1; ++a2)
            for (int v = 0; v < nv; ++v) Jx[a1][a2][v] = Jy[a1][a2][v] = 0.0;
    for (int side = 0; side < 2; ++side) {
        /* vertical face at the left (0) / right (1) of the cell */
        int64_t jx = nbr(ix + (side ? 1 : -1), C->nx, P->bc[0] == DGREF_PERIODIC);
        double x = P->xlo + (side ? ix + 1 : ix) * C->hx;
        for (int cy = 0; cy < 2; ++cy) {
            double y = P->ylo + (jy + cy) * C->hy;
            for (int a1 = 0; a1 < K1; ++a1)
                for (int a2 = 0; a2 < K1; ++a2) {
                    double din[MAXV], dout[MAXV], jmp[MAXV];
                    corner_deriv(C, u, ix, jy, a1, a2, side, cy, din);
                    if (jx >= 0) {
                        corner_deriv(C, u, jx, jy, a1, a2, 1 - side, cy, dout);
                        for (int v = 0; v < nv; ++v) jmp[v] = fabs(dout[v] - din[v]);
                    } else {
                        ghost_jump2d(P, side, x, y, t, a1, a2, din, jmp);
                    }
                    for (int v = 0; v < nv; ++v) Jx[a1][a2][v] += 0.5 * jmp[v];
                }
        }
        /* horizontal face below (0) / above (1) the cell */
        int64_t jj = nbr(jy + (side ? 1 : -1), C->ny, P->bc[2] == DGREF_PERIODIC);
        double yf = P->ylo + (side ? jy + 1 : jy) * C->hy;
        for (int cx = 0; cx < 2; ++cx) {
            double xc = P->xlo + (ix + cx) * C->hx;
            for (int a1 = 0; a1 < K1; ++a1)
                for (int a2 = 0; a2 < K1; ++a2) {
                    double din[MAXV], dout[MAXV], jmp[MAXV];
                    corner_deriv(C, u, ix, jy, a1, a2, cx, side, din);
                    if (jj >= 0) {
                        corner_deriv(C, u, ix, jj, a1, a2, cx, 1 - side, dout);
                        for (int v = 0; v < nv; ++v) jmp[v] = fabs(dout[v] - din[v]);
                    } else {
                        ghost_jump2d(P, 2 + side, xc, yf, t, a1, a2, din, jmp);
                    }
                    for (int v = 0; v < nv; ++v) Jy[a1][a2][v] += 0.5 * jmp[v];
                }
        }
    }
}

/* Damping exponents of one cell for every mode (p, q) (Sec. 2.3, mode-
 * dependent coefficient (para:damp22d)-(para:damp22d1); systems Sec. 2.4:
 * max over components; Euler: (c_fx, c_fy) = (m_x beta_x, m_y beta_y) /
 * (4 lambda_pq H-bar)).  The mesh factors (m_x, m_y) are (h_x, h_y) as
 * printed in Sec. 2.4 (cf_reading 0), (h_y, h_x) as printed for the Euler
 * examples of Sec. 3.2 (cf_reading 1; the two agree on square cells), or
 * (1, 1) (cf_reading 2, with which the 2D filter of a state varying along
 * one axis on square cells is exactly the 1D filter).  Reading for Q^k:
 * the sums over |alpha| = m run over alpha1, alpha2 <= k.  Em[m] receives
 * the exponent of mode index m; eta the hybrid indicator (Reading:
 * Jx/(2hx) + Jy/(2hy), max over components, which reduces to Algorithm 1's
 * indicator for data varying along one axis only). */
static void cell_exponents(const ctx2d* C, double t, double dt, const double* u, int64_t ix,
                           int64_t jy, double* Em, double* eta)
{
    const dgref_problem2d* P = C->P;
    const int K1 = C->K1, nv = C->nv, k = C->k;
    double Jx[MAXK + 1][MAXK + 1][MAXV], Jy[MAXK + 1][MAXK + 1][MAXV];
    cell_jumps(C, t, u, ix, jy, Jx, Jy);
    double ub[MAXV];
    for (int v = 0; v < nv; ++v) ub[v] = U(C, u, v, 0, ix, jy);
    double bx = lambda2d(P, 0, ub), by = lambda2d(P, 1, ub);
    double H = enthalpy2d(P, ub);
    for (int p = 0; p < K1; ++p)
        for (int q = 0; q < K1; ++q) {
            int l = p + q;
            if (l == 0) {
                Em[0] = 0.0;
                continue;
            }
            double lam = p * (p + 1.0) + q * (q + 1.0);
            double mx = P->cf_reading == 0 ? C->hx : P->cf_reading == 1 ? C->hy : 1.0;
            double my = P->cf_reading == 0 ? C->hy : P->cf_reading == 1 ? C->hx : 1.0;
            double cfx = mx * bx / (4.0 * lam * H);
            double cfy = my * by / (4.0 * lam * H);
            double sig = 0.0;
            for (int v = 0; v < nv; ++v) {
                double sx = C->hx * Jx[0][0][v], sy = C->hy * Jy[0][0][v];
                for (int m = 1; m <= l; ++m) {
                    double ax = 0.0, ay = 0.0;
                    for (int a1 = 0; a1 <= m && a1 <= k; ++a1) {
                        int a2 = m - a1;
                        if (a2 > k) continue;
                        ax += Jx[a1][a2][v];
                        ay += Jy[a1][a2][v];
                    }
                    sx += m * (m + 1.0) * pow(C->hx, m + 1) * ax;
                    sy += m * (m + 1.0) * pow(C->hy, m + 1) * ay;
                }
                double s = cfx * sx + cfy * sy;
                if (v == 0 || s > sig) sig = s;
            }
            double sigma = sig * (2.0 / C->hx) * (2.0 / C->hy) * lam;
            Em[p * K1 + q] = sigma * dt;
        }
    if (eta) {
        double e = 0.0;
        for (int v = 0; v < nv; ++v) {
            double ev = Jx[0][0][v] / (2.0 * C->hx) + Jy[0][0][v] / (2.0 * C->hy);
            if (v == 0 || ev > e) e = ev;
        }
        *eta = e;
    }
}

/* E[cell*(2k+1) + l]: exponent of the modes with p + q = l (taken from the
 * mode (l - q, q) with the smallest admissible q); eta[cell]. */
int dgref_exponents2d(const dgref_problem2d* P, double t, double dt, const double* v, double* E,
                      double* eta)
{
    ctx2d C;
    int rc = make_ctx(P, &C);
    if (rc) return rc;
    const int L1 = 2 * C.k + 1;
#pragma omp parallel for schedule(static) if (C.nx * C.ny >= 4096)
    for (int64_t jy = 0; jy < C.ny; ++jy)
        for (int64_t ix = 0; ix < C.nx; ++ix) {
            double Em[NMAX], e;
            cell_exponents(&C, t, dt, v, ix, jy, Em, &e);
            size_t cell = (size_t)jy * C.nx + ix;
            for (int l = 0; l < L1; ++l) {
                int q = l > C.k ? l - C.k : 0;
                E[cell * L1 + l] = Em[(l - q) * C.K1 + q];
            }
            if (eta) eta[cell] = e;
        }
    return DGREF_OK;
}

/* Post-stage operator (jump filter / hybrid, Algorithm 1) at time t. */
int dgref_post2d(const dgref_problem2d* P, int stage, double t, double dt, const double* v,
                 double* out, int64_t* troubled)
{
    static const double stage_weight[3] = {1.0, 0.25, 2.0 / 3.0};
    ctx2d C;
    int rc = make_ctx(P, &C);
    if (rc) return rc;
    const size_t ncell = (size_t)C.nx * C.ny;
    const size_t ndof = (size_t)C.nv * C.NM * ncell;
    if (P->filter == DGREF_FILTER_NONE) {
        if (out != v) memcpy(out, v, sizeof(double) * ndof);
        return P->pp ? dgref_pp_limit2d(P, out) : DGREF_OK;
    }
    double tau = (P->filter_dt == 1) ? dt * stage_weight[stage] : dt;
    double* Em = (double*)malloc(sizeof(double) * ncell * C.NM);
    double* eta = (double*)malloc(sizeof(double) * ncell);
    if (!Em || !eta) {
        free(Em);
        free(eta);
        return DGREF_ERR_ARG;
    }
#pragma omp parallel for schedule(static) if (C.nx * C.ny >= 4096)
    for (int64_t jy = 0; jy < C.ny; ++jy)
        for (int64_t ix = 0; ix < C.nx; ++ix) {
            size_t cell = (size_t)jy * C.nx + ix;
            cell_exponents(&C, t, tau, v, ix, jy, Em + cell * C.NM, eta + cell);
        }
    double M = 0.0;
    for (size_t c = 0; c < ncell; ++c)
        if (!(eta[c] <= M)) M = eta[c];
    int64_t cnt = 0;
    for (int64_t jy = 0; jy < C.ny; ++jy)
        for (int64_t ix = 0; ix < C.nx; ++ix) {
            size_t cell = (size_t)jy * C.nx + ix;
            int hybrid = P->filter == DGREF_FILTER_HYBRID;
            int hit = hybrid ? eta[cell] > 1.0 : 1;
            double w = (hybrid && hit) ? (M - eta[cell]) / (M - 1.0) : 0.0;
            if (hybrid) cnt += hit;
            for (int var = 0; var < C.nv; ++var)
                for (int m = 0; m < C.NM; ++m) {
                    double dg = U(&C, v, var, m, ix, jy);
                    double r = dg;
                    if (hit && m > 0) {
                        double lim = exp(-Em[cell * C.NM + m]) * dg;
                        r = hybrid ? w * dg + (1.0 - w) * lim : lim;
                    }
                    *Up(&C, out, var, m, ix, jy) = r;
                }
        }
    if (troubled) *troubled += cnt;
    free(Em);
    free(eta);
    return P->pp ? dgref_pp_limit2d(P, out) : DGREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Positivity-preserving limiter on rectangles (Zhang and Shu; the paper     */
/* applies it after the jump filter in its Sec. 3.2 examples with extreme    */
/* positivity demands)                                                       */
/* ------------------------------------------------------------------------ */

/* Test points: the tensor sets (Gauss-Lobatto in xi) x (Gauss in eta) and
 * (Gauss in xi) x (Gauss-Lobatto in eta), with N = ceil((k+3)/2) Lobatto
 * points (the ends +-1 and, for N = 3, the centre 0): the Q^k cell average
 * is a convex combination of the values there, and they contain the edge
 * Gauss points where the fluxes are evaluated.  The Gauss x Gauss points of
 * the volume quadrature are added, so the volume fluxes also see admissible
 * states.  px[i][p] = P_p(xi_i), py[i][q] = P_q(eta_i), taken from the
 * tables the DG operator uses, so a value here is bitwise the value the
 * fluxes see. */
static int pp_tables2d(const ctx2d* C, double px[][MAXK + 1], double py[][MAXK + 1], double* xi,
                       double* eta)
{
    const int K1 = C->K1, nq = C->B.nq;
    const int N = (C->k + 4) / 2 < 2 ? 2 : (C->k + 4) / 2;
    double gl[3][MAXK + 1], glx[3];
    for (int l = 0; l < K1; ++l) {
        gl[0][l] = C->B.tr[0][l][0];
        gl[1][l] = C->B.tr[1][l][0];
        gl[2][l] = dgref_legendre_deriv(l, 0, 0.0);
    }
    glx[0] = -1.0;
    glx[1] = 1.0;
    glx[2] = 0.0;
    int cnt = 0;
    for (int dir = 0; dir < 2; ++dir)
        for (int i = 0; i < N; ++i)
            for (int b = 0; b < nq; ++b, ++cnt) {
                const double* lob = gl[i];
                const double* gau = C->B.phi[b];
                for (int l = 0; l < K1; ++l) {
                    px[cnt][l] = dir == 0 ? lob[l] : gau[l];
                    py[cnt][l] = dir == 0 ? gau[l] : lob[l];
                }
                if (xi) xi[cnt] = dir == 0 ? glx[i] : C->B.xq[b];
                if (eta) eta[cnt] = dir == 0 ? C->B.xq[b] : glx[i];
            }
    for (int a = 0; a < nq; ++a)
        for (int b = 0; b < nq; ++b, ++cnt) {
            for (int l = 0; l < K1; ++l) {
                px[cnt][l] = C->B.phi[a][l];
                py[cnt][l] = C->B.phi[b][l];
            }
            if (xi) xi[cnt] = C->B.xq[a];
            if (eta) eta[cnt] = C->B.xq[b];
        }
    return cnt;
}

int dgref_pp_points2d(const dgref_problem2d* P, double* xi, double* eta)
{
    ctx2d C;
    int rc = make_ctx(P, &C);
    if (rc) return rc;
    double px[PPMAX][MAXK + 1], py[PPMAX][MAXK + 1];
    return pp_tables2d(&C, px, py, xi, eta);
}

static double pressure_pp2d(double gamma, const double* w)
{
    return (gamma - 1.0) * (w[3] - 0.5 * (w[1] * w[1] + w[2] * w[2]) / w[0]);
}

/* The pressure as the flux and the wave speed evaluate it (flux2d). */
static double pressure_flux_pp2d(double gamma, const double* w)
{
    const double vx = w[1] / w[0], vy = w[2] / w[0];
    return (gamma - 1.0) * (w[3] - 0.5 * (w[1] * vx + w[2] * vy));
}

/* Point value w and the sums wa of the magnitudes of its terms. */
static void point_value_abs(const ctx2d* C, const double* u, int64_t ix, int64_t jy,
                            const double* px, const double* py, double* w, double* wa)
{
    for (int v = 0; v < 4; ++v) {
        double s = 0.0, sa = 0.0;
        for (int p = 0; p < C->K1; ++p)
            for (int q = 0; q < C->K1; ++q) {
                const double term = U(C, u, v, p * C->K1 + q, ix, jy) * px[p] * py[q];
                s += term;
                sa += fabs(term);
            }
        w[v] = s;
        wa[v] = sa;
    }
}

/* Limit cell (ix, jy) in place, as the 1D limiter does: scale the density's
 * higher modes so the density at every test point is >= eps_r, then all
 * higher modes so the pressure at each point is >= eps_p (bisection for the
 * largest t in [0,1] with p(u_bar + t (u(x) - u_bar)) >= eps_p; p is concave
 * along the segment); eps = min(1e-13, rho_bar, p(u_bar)), raised per point
 * to its rounding margin (8 units of roundoff times the magnitudes that
 * cancel), which vanishes in exact arithmetic.  The scaled cell is then
 * checked in the fluxes' own arithmetic, its higher modes halved until the
 * density and pressure are positive at every point (dropped after 50
 * halvings).  Cell averages are not changed. */
static void pp_limit_cell2d(const ctx2d* C, double* u, int64_t ix, int64_t jy, int np,
                            double px[][MAXK + 1], double py[][MAXK + 1])
{
    const double gamma = C->P->gamma, ur = 0x1p-52;
    double ub[4];
    for (int v = 0; v < 4; ++v) ub[v] = U(C, u, v, 0, ix, jy);
    const double pb = pressure_pp2d(gamma, ub);
    if (!(ub[0] > 0.0) || !(pb > 0.0)) return; /* inadmissible average: not limitable */
    double eps = 1e-13;
    if (ub[0] < eps) eps = ub[0];
    if (pb < eps) eps = pb;
    /* density */
    double rmin = INFINITY, eps_r = eps;
    for (int i = 0; i < np; ++i) {
        double w[4], wa[4];
        point_value_abs(C, u, ix, jy, px[i], py[i], w, wa);
        if (w[0] < rmin) rmin = w[0];
        if (8.0 * ur * wa[0] > eps_r) eps_r = 8.0 * ur * wa[0];
    }
    if (eps_r > ub[0]) eps_r = ub[0];
    if (rmin < eps_r) {
        double th = (ub[0] - eps_r) / (ub[0] - rmin);
        if (th < 0.0) th = 0.0;
        for (int m = 1; m < C->NM; ++m) *Up(C, u, 0, m, ix, jy) *= th;
    }
    /* pressure */
    double theta = 1.0;
    for (int i = 0; i < np; ++i) {
        double w[4], wa[4];
        point_value_abs(C, u, ix, jy, px[i], py[i], w, wa);
        double eps_p = eps;
        if (w[0] > 0.0) {
            const double kin = 0.5 * (w[1] * w[1] + w[2] * w[2]) / w[0];
            const double m = 8.0 * ur *
                             (wa[3] + (fabs(w[1]) * wa[1] + fabs(w[2]) * wa[2]) / w[0] +
                              kin * wa[0] / w[0]);
            if (m > eps_p) eps_p = m;
        }
        if (eps_p > pb) eps_p = pb;
        if (pressure_pp2d(gamma, w) >= eps_p) continue;
        double lo = 0.0, hi = 1.0;
        for (int it = 0; it < 60; ++it) {
            double mid = 0.5 * (lo + hi), wm[4];
            for (int v = 0; v < 4; ++v) wm[v] = ub[v] + mid * (w[v] - ub[v]);
            if (pressure_pp2d(gamma, wm) >= eps_p)
                lo = mid;
            else
                hi = mid;
        }
        if (lo < theta) theta = lo;
    }
    if (theta < 1.0)
        for (int v = 0; v < 4; ++v)
            for (int m = 1; m < C->NM; ++m) *Up(C, u, v, m, ix, jy) *= theta;
    /* positivity in the fluxes' own arithmetic */
    for (int halving = 0; halving <= 50; ++halving) {
        int ok = 1;
        for (int i = 0; i < np && ok; ++i) {
            double w[4];
            point_value(C, u, ix, jy, px[i], py[i], w);
            ok = w[0] > 0.0 && pressure_flux_pp2d(gamma, w) > 0.0;
        }
        if (ok) return;
        const double f = halving < 50 ? 0.5 : 0.0;
        for (int v = 0; v < 4; ++v)
            for (int m = 1; m < C->NM; ++m) *Up(C, u, v, m, ix, jy) *= f;
    }
}

int dgref_pp_limit2d(const dgref_problem2d* P, double* u)
{
    ctx2d C;
    int rc = make_ctx(P, &C);
    if (rc) return rc;
    if (P->eq != DGREF_EULER) return DGREF_OK;
    double px[PPMAX][MAXK + 1], py[PPMAX][MAXK + 1];
    const int np = pp_tables2d(&C, px, py, NULL, NULL);
#pragma omp parallel for schedule(static) if (C.nx * C.ny >= 4096)
    for (int64_t jy = 0; jy < C.ny; ++jy)
        for (int64_t ix = 0; ix < C.nx; ++ix) pp_limit_cell2d(&C, u, ix, jy, np, px, py);
    return DGREF_OK;
}

static int averages_admissible2d(const ctx2d* C, const double* u)
{
    for (int64_t jy = 0; jy < C->ny; ++jy)
        for (int64_t ix = 0; ix < C->nx; ++ix) {
            double w[4];
            for (int v = 0; v < 4; ++v) w[v] = U(C, u, v, 0, ix, jy);
            if (!(w[0] > 0.0) || !(pressure_pp2d(C->P->gamma, w) > 0.0)) return 0;
        }
    return 1;
}

/* One SSP-RK3 step from time t with the post-stage operator after every
 * stage; the filter after stage s uses the time its output stands for,
 * t + (1, 1/2, 1)[s] dt, for time-dependent boundary states.  With the
 * positivity limiter a rejected step returns DGREF_ERR_POSITIVITY and leaves
 * u and troubled untouched. */
int dgref_step2d(const dgref_problem2d* P, double t, double dt, double* u, int64_t* troubled)
{
    static const double cf[3] = {1.0, 0.5, 1.0};
    ctx2d C;
    int rc = make_ctx(P, &C);
    if (rc) return rc;
    const size_t ndof = (size_t)C.nv * C.NM * C.nx * C.ny;
    double* un = (double*)malloc(sizeof(double) * ndof);
    double* us = (double*)malloc(sizeof(double) * ndof);
    double* w = (double*)malloc(sizeof(double) * ndof);
    if (!un || !us || !w) {
        rc = DGREF_ERR_ARG;
        goto done;
    }
    memcpy(un, u, sizeof(double) * ndof);
    memcpy(us, u, sizeof(double) * ndof);
    const int64_t tr0 = troubled ? *troubled : 0;
    for (int s = 0; s < 3 && !rc; ++s) {
        rc = dgref_stage2d(P, s, t, dt, un, us, w);
        if (!rc) rc = dgref_post2d(P, s, t + cf[s] * dt, dt, w, us, troubled);
        /* positivity limiter: a stage whose cell averages leave the
         * admissible set rejects the step (u untouched; retried by the
         * caller with a smaller dt) */
        if (!rc && P->pp && !averages_admissible2d(&C, us)) rc = DGREF_ERR_POSITIVITY;
    }
    if (!rc) memcpy(u, us, sizeof(double) * ndof);
    else if (troubled) *troubled = tr0;
done:
    free(un);
    free(us);
    free(w);
    return rc;
}

/* Density and pressure at every volume and edge Gauss point (Euler) and
 * finiteness of every coefficient. */
int dgref_check2d(const dgref_problem2d* P, const double* u, double* min_rho, double* min_p,
                  int64_t* first_bad)
{
    ctx2d C;
    int rc = make_ctx(P, &C);
    if (rc) return rc;
    double mr = INFINITY, mp = INFINITY;
    int status = DGREF_OK;
    int64_t bad = -1;
    const int nq = C.B.nq, K1 = C.K1;
    for (int64_t jy = 0; jy < C.ny; ++jy)
        for (int64_t ix = 0; ix < C.nx; ++ix) {
            int64_t cell = jy * C.nx + ix;
            int finite = 1;
            for (int v = 0; v < C.nv; ++v)
                for (int m = 0; m < C.NM; ++m)
                    if (!isfinite(U(&C, u, v, m, ix, jy))) finite = 0;
            if (!finite) {
                if (status == DGREF_OK) {
                    status = DGREF_ERR_NONFINITE;
                    bad = cell;
                }
                continue;
            }
            if (P->eq != DGREF_EULER) continue;
            for (int a = 0; a < nq + 2; ++a)
                for (int b = 0; b < nq + 2; ++b) {
                    if (a >= nq && b >= nq) continue; /* corners are not checked */
                    double px[MAXK + 1], py[MAXK + 1], uq[MAXV];
                    for (int p = 0; p < K1; ++p) px[p] = a < nq ? C.B.phi[a][p] : C.B.tr[a - nq][p][0];
                    for (int q = 0; q < K1; ++q) py[q] = b < nq ? C.B.phi[b][q] : C.B.tr[b - nq][q][0];
                    point_value(&C, u, ix, jy, px, py, uq);
                    double p = pressure2d(P, uq);
                    if (uq[0] < mr) mr = uq[0];
                    if (p < mp) mp = p;
                    if ((!(uq[0] > 0.0) || !(p > 0.0)) && status == DGREF_OK && !P->pp) {
                        status = DGREF_ERR_POSITIVITY;
                        bad = cell;
                    }
                }
            /* with the positivity limiter, point values sit at its margin
             * up to rounding: only an inadmissible cell average is an error */
            if (P->pp && status == DGREF_OK) {
                double w[4];
                for (int v = 0; v < 4; ++v) w[v] = U(&C, u, v, 0, ix, jy);
                if (!(w[0] > 0.0) || !(pressure2d(P, w) > 0.0)) {
                    status = DGREF_ERR_POSITIVITY;
                    bad = cell;
                }
            }
        }
    if (min_rho) *min_rho = mr;
    if (min_p) *min_p = mp;
    if (first_bad) *first_bad = bad;
    return status;
}

/* Time loop: dt = cfl / max(lambda_x/hx + lambda_y/hy), the last step
 * clamped to end exactly at t_end. */
int dgref_run2d(const dgref_problem2d* P, double t_end, int64_t max_steps, double* u,
                dgref_report* rep)
{
    ctx2d C;
    int rc = make_ctx(P, &C);
    if (rc) return rc;
    dgref_report r;
    memset(&r, 0, sizeof r);
    r.dt_min = INFINITY;
    r.first_bad_cell = -1;
    double t = 0.0;
    while (t < t_end && r.steps < max_steps) {
        double alpha = dgref_max_wavespeed2d(P, u);
        if (!isfinite(alpha)) {
            rc = DGREF_ERR_NONFINITE;
            break;
        }
        double dt = P->cfl / alpha;
        int last = 0;
        if (t + dt >= t_end) {
            dt = t_end - t;
            last = 1;
        }
        rc = dgref_step2d(P, t, dt, u, &r.troubled_cells);
        /* positivity limiter: a rejected step is retried with half the time
         * step (Zhang and Shu's remedy when a stage violates the CFL bound
         * of the positivity argument) */
        for (int tries = 0; rc == DGREF_ERR_POSITIVITY && P->pp && tries < DGREF_MAX_RETRIES;
             ++tries) {
            dt *= 0.5;
            last = 0;
            r.restarts++;
            rc = dgref_step2d(P, t, dt, u, &r.troubled_cells);
        }
        if (rc) break;
        t = last ? t_end : t + dt;
        r.steps++;
        if (dt < r.dt_min) r.dt_min = dt;
        if (dt > r.dt_max) r.dt_max = dt;
    }
    r.t = t;
    for (int v = 0; v < C.nv; ++v) {
        double q = 0.0;
        for (int64_t jy = 0; jy < C.ny; ++jy)
            for (int64_t ix = 0; ix < C.nx; ++ix) q += C.hx * C.hy * U(&C, u, v, 0, ix, jy);
        r.ledger[v] = q;
    }
    int crc = dgref_check2d(P, u, &r.min_rho, &r.min_p, &r.first_bad_cell);
    if (!rc) rc = crc;
    r.status = rc;
    if (rep) *rep = r;
    return rc;
}
