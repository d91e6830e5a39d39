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

#endif
