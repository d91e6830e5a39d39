/* dgref_internal.h — tables shared by the 1D and 2D parts of the oracle
 * (test infrastructure only). */
#ifndef DGREF_INTERNAL_H
#define DGREF_INTERNAL_H

#define MAXK 4
#define MAXQ 8
#define MAXV 4

typedef struct {
    int k, nq;
    double xq[MAXQ], wq[MAXQ];
    double phi[MAXQ][MAXK + 1];       /* P_l(xi_q)                         */
    double dphi[MAXQ][MAXK + 1];      /* P_l'(xi_q)                        */
    double tr[2][MAXK + 1][MAXK + 1]; /* tr[side][l][m] = P_l^(m)(-1 / +1) */
} dgref_basis;

int dgref_make_basis(int k, int nq, dgref_basis* B);

/* HLL (kind 1) / HLLC (kind 2) Euler flux across a face of normal `dir`
 * (dgref_hll.c); nv = 3 (1D) or 4 (2D). */
void dgref_hll_flux(int kind, int nv, int dir, double gamma, const double* UL, const double* UR,
                    double* F);

#endif
