/* dgref_hll.c — HLL and HLLC numerical fluxes of the Euler equations for
 * the oracle (test infrastructure; plain FP64).
 *
 * The paper's computations use the local Lax-Friedrichs flux; Sec. 3 names
 * HLL (Harten, Lax and van Leer) and HLLC (Harten-Lax-van Leer-Contact, as
 * in Toro's textbook) as alternatives that work with the filter.  The paper
 * gives no formulas, so these follow the textbook statements in primitive
 * variables:
 *   - wave-speed bounds (Davis): S_L = min(u_L - a_L, u_R - a_R),
 *     S_R = max(u_L + a_L, u_R + a_R), a = sqrt(gamma p / rho);
 *   - HLL: F = F_L if 0 <= S_L, F_R if S_R <= 0, else
 *     (S_R F_L - S_L F_R + S_L S_R (U_R - U_L)) / (S_R - S_L);
 *   - HLLC: middle wave
 *     S* = (p_R - p_L + rho_L u_L (S_L - u_L) - rho_R u_R (S_R - u_R))
 *          / (rho_L (S_L - u_L) - rho_R (S_R - u_R)),
 *     star states U*_K = rho_K (S_K - u_K)/(S_K - S*) *
 *       [1, S*, (v_K), E_K/rho_K + (S* - u_K)(S* + p_K/(rho_K (S_K - u_K)))],
 *     F = F_L, F_L + S_L (U*_L - U_L), F_R + S_R (U*_R - U_R), F_R on the four
 *     sides of 0 among S_L <= S* <= S_R.
 * The state is (rho, momentum..., E) with `nv` = 3 (1D) or 4 (2D); `dir`
 * picks the normal momentum (0: x, 1: y), the other one is tangential.
 * fmin / fmax take the bound from the other state when a sound speed is NaN
 * (an inadmissible state with negative pressure). */
#include <math.h>

#include "dgref_internal.h"

typedef struct {
    double rho, un, ut, E, p, a;
} prim;

static prim primitive(int nv, int dir, double gamma, const double* U)
{
    prim w;
    w.rho = U[0];
    const double mx = U[1], my = nv == 4 ? U[2] : 0.0;
    w.E = U[nv - 1];
    const double ux = mx / w.rho, uy = my / w.rho;
    w.un = dir == 0 ? ux : uy;
    w.ut = dir == 0 ? uy : ux;
    w.p = (gamma - 1.0) * (w.E - 0.5 * w.rho * (ux * ux + uy * uy));
    w.a = sqrt(gamma * w.p / w.rho);
    return w;
}

/* Physical normal flux of state U. */
static void normal_flux(int nv, int dir, const prim* w, const double* U, double* F)
{
    F[0] = w->rho * w->un;
    for (int v = 1; v < nv - 1; ++v) F[v] = U[v] * w->un;
    F[1 + dir] += w->p;
    F[nv - 1] = (w->E + w->p) * w->un;
}

void dgref_hll_flux(int kind, int nv, int dir, double gamma, const double* UL, const double* UR,
                    double* F)
{
    const prim L = primitive(nv, dir, gamma, UL), R = primitive(nv, dir, gamma, UR);
    double FL[4], FR[4];
    normal_flux(nv, dir, &L, UL, FL);
    normal_flux(nv, dir, &R, UR, FR);
    const double SL = fmin(L.un - L.a, R.un - R.a);
    const double SR = fmax(L.un + L.a, R.un + R.a);
    if (SL >= 0.0) {
        for (int v = 0; v < nv; ++v) F[v] = FL[v];
        return;
    }
    if (SR <= 0.0) {
        for (int v = 0; v < nv; ++v) F[v] = FR[v];
        return;
    }
    if (kind == 1) { /* HLL */
        for (int v = 0; v < nv; ++v)
            F[v] = (SR * FL[v] - SL * FR[v] + SL * SR * (UR[v] - UL[v])) / (SR - SL);
        return;
    }
    /* HLLC */
    const double Sstar = (R.p - L.p + L.rho * L.un * (SL - L.un) - R.rho * R.un * (SR - R.un)) /
                         (L.rho * (SL - L.un) - R.rho * (SR - R.un));
    const prim* K = Sstar >= 0.0 ? &L : &R;
    const double* UK = Sstar >= 0.0 ? UL : UR;
    const double* FK = Sstar >= 0.0 ? FL : FR;
    const double SK = Sstar >= 0.0 ? SL : SR;
    const double scale = K->rho * (SK - K->un) / (SK - Sstar);
    double Us[4];
    Us[0] = scale;
    if (nv == 4) {
        Us[1 + dir] = scale * Sstar;
        Us[2 - dir] = scale * K->ut;
    } else {
        Us[1] = scale * Sstar;
    }
    Us[nv - 1] = scale * (K->E / K->rho + (Sstar - K->un) * (Sstar + K->p / (K->rho * (SK - K->un))));
    for (int v = 0; v < nv; ++v) F[v] = FK[v] + SK * (Us[v] - UK[v]);
}
