/* ADG oracle — test infrastructure only.  Internal declarations of the oracle. */
#ifndef ADG_OR_INTERNAL_H
#define ADG_OR_INTERNAL_H

#include "oracle.h"

#define OR_MAXNS 16
#define OR_MAXV (3 + OR_MAXNS)
#define OR_MAXM 6
#define OR_MAXQ 10
#define OR_MAXR 64

/* Primitive state at one point. */
typedef struct {
  double rho, u, p, T, a;
  double Y[OR_MAXNS];
  /* detailed model only */
  double cp, cv;                 /* mixture, J/(kg K) */
  double e_sp[OR_MAXNS];         /* species internal energy, J/kg */
  double h_sp[OR_MAXNS];         /* species enthalpy, J/kg */
} or_prim;

int or_primitives(const or_config *cfg, const double *w, or_prim *pr);
void or_flux_from_prim(const or_config *cfg, const double *w, const or_prim *pr, double *f);
int or_source_from_prim(const or_config *cfg, const double *w, const or_prim *pr, double *s);
void or_diff_flux_from_prim(const or_config *cfg, const double *w, const or_prim *pr,
                            const double *dwdx, double *fd);

/* Monomial coefficients of the Legendre polynomial P_j (ascending powers). */
void or_legendre_monomial(int j, double *c);

/* Solve the dense n x n system A x = b by Gauss-Jordan with partial pivoting
   (A and b are overwritten).  Returns 0 on success. */
int or_dense_solve(int n, double *A, double *b, int nrhs);

#endif
