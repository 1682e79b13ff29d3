/*
 * ADG oracle — test infrastructure only.
 *
 * The limiter of Sec. 3.3: characteristic decomposition of the flux Jacobian
 * A = R Lambda L at the cell mean, the simple WENO reconstruction of Eq. (9)-(10)
 * on characteristic variables, and the KXRCF troubled-cell indicator.
 * The asynchrony-tolerant neighbour data of Eq. (11) is supplied by the caller
 * (or_solver.c), so the same cell routine serves WENO and AT-WENO.
 *
 * Readings (the paper is silent or garbled here):
 *   * Eigenvectors: only Lambda = diag(u-a, u, .., u, u+a) is given.  Rows of L:
 *       (dp - rho a du)/(2a^2), drho - dp/a^2, d(rho Y_i) - Y_i drho (i < Ns-1),
 *       d(sum_i rho Y_i - rho), (dp + rho a du)/(2a^2),
 *     each a linear form in the conserved variables at the mean state; R = L^-1.
 *     The fourth kind keeps sum_i rho Y_i = rho through the limiter.
 *   * In the tilde form of Eq. (9) the neighbour mean that is replaced is the
 *     neighbour polynomial's mean over the cell itself, so the limited cell
 *     keeps its mean; neighbours are re-expanded in the cell's coordinate.
 *   * Eq. (10)'s integral is over the cell for all three candidates; mapped to
 *     the reference coordinate it is the constant quadratic form
 *     B_ab = sum_{s=1..Np} 2^(2s-1) int P_a^(s) P_b^(s) dxi.
 *   * The combination is convex (positive weights summing to one).
 *   * Troubled cells: KXRCF (Krivodonova et al. 2004) on rho and rho E in place
 *     of the paper's TVD indicator.
 *
 * Pins (tests/test_oracle_limiter.py): B against numpy polynomial integration,
 * translation against numpy polynomial evaluation, L A R = Lambda with A by
 * finite differences, cell means preserved, a global polynomial reproduced,
 * smooth data not flagged, a jump flagged.
 */
#include <math.h>
#include <string.h>

#include "or_internal.h"

/* Rows of L at the mean state wbar (one-step model), R = L^-1.  Row-major V x V. */
int or_char_matrices(const or_config *cfg, const double *wbar, double *Lm, double *Rm) {
  int ns = cfg->n_species, V = 3 + ns;
  if (cfg->model != OR_ONESTEP) return -1;
  or_prim pr;
  if (or_primitives(cfg, wbar, &pr)) return -1;
  double rho = pr.rho, u = pr.u, a = pr.a, g1 = cfg->gamma - 1.0;
  double dp[OR_MAXV] = {0}, du[OR_MAXV] = {0}, drho[OR_MAXV] = {0};
  dp[0] = g1 * 0.5 * u * u;
  dp[1] = -g1 * u;
  dp[2] = g1;
  dp[3] = -g1 * cfg->q_heat;
  du[0] = -u / rho;
  du[1] = 1.0 / rho;
  drho[0] = 1.0;
  memset(Lm, 0, sizeof(double) * V * V);
  for (int c = 0; c < V; ++c) {
    Lm[0 * V + c] = (dp[c] - rho * a * du[c]) / (2.0 * a * a);
    Lm[1 * V + c] = drho[c] - dp[c] / (a * a);
    Lm[(V - 1) * V + c] = (dp[c] + rho * a * du[c]) / (2.0 * a * a);
  }
  for (int i = 0; i < ns - 1; ++i) {
    Lm[(2 + i) * V + 0] = -pr.Y[i];
    Lm[(2 + i) * V + 3 + i] = 1.0;
  }
  Lm[(V - 2) * V + 0] = -1.0;
  for (int i = 0; i < ns; ++i) Lm[(V - 2) * V + 3 + i] = 1.0;
  /* R = L^-1 */
  double A[OR_MAXV * OR_MAXV];
  memcpy(A, Lm, sizeof(double) * V * V);
  memset(Rm, 0, sizeof(double) * V * V);
  for (int i = 0; i < V; ++i) Rm[i * V + i] = 1.0;
  return or_dense_solve(V, A, Rm, V);
}

/* Smoothness-indicator quadratic form of Eq. (10) in reference coordinates. */
void or_beta_matrix(int np, double *B) {
  int M = np + 1;
  double x[OR_MAXQ], w[OR_MAXQ];
  or_gauss_legendre(M, x, w);
  for (int a = 0; a < M; ++a)
    for (int b = 0; b < M; ++b) {
      double sum = 0.0;
      for (int s = 1; s <= np; ++s) {
        double integral = 0.0;
        for (int q = 0; q < M; ++q)
          integral += w[q] * or_legendre_deriv(a, s, x[q]) * or_legendre_deriv(b, s, x[q]);
        sum += ldexp(1.0, 2 * s - 1) * integral;
      }
      B[a * M + b] = sum;
    }
}

/* Modal coefficients, in the cell's own coordinate xi, of the neighbour on side
   `side` (+1 right, -1 left) extended over the cell: the neighbour's coordinate
   is xi - 2 side.  T[k][j] is the L2 projection of P_j(xi - 2 side) onto P_k. */
void or_translation(int np, int side, double *T) {
  int M = np + 1;
  double x[OR_MAXQ], w[OR_MAXQ];
  or_gauss_legendre(M + 1, x, w);
  for (int k = 0; k < M; ++k) {
    double mkk = 0.0;
    for (int q = 0; q < M + 1; ++q) mkk += w[q] * or_legendre(k, x[q]) * or_legendre(k, x[q]);
    for (int j = 0; j < M; ++j) {
      double s = 0.0;
      for (int q = 0; q < M + 1; ++q) s += w[q] * or_legendre(j, x[q] - 2.0 * side) * or_legendre(k, x[q]);
      T[k * M + j] = s / mkk;
    }
  }
}

/* WENO limiting of one cell from the (unlimited) modal data of its stencil.
   wl, wc, wr, out: [V][M].  Eq. (9)-(10) on characteristic variables. */
int or_weno_cell(const or_config *cfg, const double *wl, const double *wc, const double *wr, double *out) {
  int V = 3 + cfg->n_species, np = cfg->order_p, M = np + 1;
  double Lm[OR_MAXV * OR_MAXV], Rm[OR_MAXV * OR_MAXV], wbar[OR_MAXV];
  for (int v = 0; v < V; ++v) wbar[v] = wc[v * M + 0];
  if (or_char_matrices(cfg, wbar, Lm, Rm)) return -1;
  double B[OR_MAXM * OR_MAXM], Tl[OR_MAXM * OR_MAXM], Tr[OR_MAXM * OR_MAXM];
  or_beta_matrix(np, B);
  or_translation(np, -1, Tl);
  or_translation(np, +1, Tr);
  const double *stencil[3] = {wl, wc, wr};
  const double *Tm[3] = {Tl, NULL, Tr};
  double vt[3][OR_MAXV][OR_MAXM];
  /* v_{e+j} = L w_{e+j}, mode by mode */
  for (int s = 0; s < 3; ++s)
    for (int c = 0; c < V; ++c)
      for (int j = 0; j < M; ++j) {
        double acc = 0.0;
        for (int v = 0; v < V; ++v) acc += Lm[c * V + v] * stencil[s][v * M + j];
        vt[s][c][j] = acc;
      }
  /* neighbours: re-expand in the cell's coordinate, then set the mean to v_e's */
  for (int s = 0; s < 3; s += 2)
    for (int c = 0; c < V; ++c) {
      double tmp[OR_MAXM];
      for (int k = 0; k < M; ++k) {
        double acc = 0.0;
        for (int j = 0; j < M; ++j) acc += Tm[s][k * M + j] * vt[s][c][j];
        tmp[k] = acc;
      }
      tmp[0] = vt[1][c][0];
      for (int k = 0; k < M; ++k) vt[s][c][k] = tmp[k];
    }
  double vlim[OR_MAXV][OR_MAXM];
  for (int c = 0; c < V; ++c) {
    double wbarj[3], sum = 0.0;
    for (int s = 0; s < 3; ++s) {
      double beta = 0.0;
      for (int a = 0; a < M; ++a)
        for (int b = 0; b < M; ++b) beta += vt[s][c][a] * B[a * M + b] * vt[s][c][b];
      double d = cfg->weno_eps + beta;
      wbarj[s] = cfg->weno_gamma[s] / (d * d);
      sum += wbarj[s];
    }
    for (int j = 0; j < M; ++j) {
      double acc = 0.0;
      for (int s = 0; s < 3; ++s) acc += (wbarj[s] / sum) * vt[s][c][j];
      vlim[c][j] = acc;
    }
  }
  /* w_lim = R v_lim */
  for (int v = 0; v < V; ++v)
    for (int j = 0; j < M; ++j) {
      double acc = 0.0;
      for (int c = 0; c < V; ++c) acc += Rm[v * V + c] * vlim[c][j];
      out[v * M + j] = acc;
    }
  return 0;
}
