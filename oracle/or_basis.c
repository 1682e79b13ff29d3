/*
 * ADG oracle — test infrastructure only.
 *
 * Modal basis and quadrature of the standard DG method (Sec. 3.1, Eq. (5)-(6)),
 * the asynchrony-tolerant weights of Eq. (7)-(8) and the delay models of
 * Sec. 4.1 (CAA) and Sec. 4.2 (SAA).
 *
 * Pins (tests/test_oracle_basis.py, tests/test_oracle_async.py):
 *   Legendre values and derivatives  -> numpy.polynomial.legendre (library routine)
 *   Gauss-Legendre nodes / weights   -> closed forms for 2 and 3 points, exactness on
 *                                       monomials, numpy.polynomial.legendre.leggauss
 *   AT weights                       -> Table 1 as printed (golden fixture, with the
 *                                       one misprinted entry documented), Eq. (8)
 *                                       residuals checked in exact rationals
 *   SplitMix64                       -> published test vector
 *   delay binning                    -> empirical frequencies vs the probability set
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "or_internal.h"

/* Legendre polynomial P_j(x), normalised with P_j(1) = 1, by Bonnet's
   three-term recurrence (j+1) P_{j+1} = (2j+1) x P_j - j P_{j-1}.
   The paper's basis phi_j is "polynomials of degree up to N_p" (Sec. 3.1); the
   Legendre choice is this solver's reading. */
double or_legendre(int j, double x) {
  if (j == 0) return 1.0;
  double p0 = 1.0, p1 = x;
  for (int k = 1; k < j; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

/* Monomial coefficients of P_j from the same recurrence, on coefficient arrays.
   For the orders used here every coefficient is a dyadic rational, so the
   arithmetic is exact. */
void or_legendre_monomial(int j, double *c) {
  double pm[OR_MAXM + 4] = {0}, pc[OR_MAXM + 4] = {0}, pn[OR_MAXM + 4];
  pm[0] = 1.0;          /* P_0 */
  if (j == 0) {
    memset(c, 0, sizeof(double) * (j + 1));
    c[0] = 1.0;
    return;
  }
  pc[1] = 1.0;          /* P_1 */
  for (int k = 1; k < j; ++k) {
    memset(pn, 0, sizeof pn);
    for (int d = 0; d <= k; ++d) pn[d + 1] += (2.0 * k + 1.0) * pc[d];
    for (int d = 0; d <= k - 1; ++d) pn[d] -= k * pm[d];
    for (int d = 0; d <= k + 1; ++d) pn[d] /= (k + 1.0);
    memcpy(pm, pc, sizeof pc);
    memcpy(pc, pn, sizeof pn);
  }
  for (int d = 0; d <= j; ++d) c[d] = pc[d];
}

/* s-th derivative of P_j at x, from the monomial form. */
double or_legendre_deriv(int j, int s, double x) {
  double c[OR_MAXM + 4];
  or_legendre_monomial(j, c);
  double r = 0.0;
  for (int d = j; d >= s; --d) {
    double fac = 1.0;
    for (int t = 0; t < s; ++t) fac *= (double)(d - t);
    r = r * x + fac * c[d];
  }
  return r;
}

/* Gauss-Legendre rule with n points on [-1, 1]: the nodes are the roots of P_n,
   found by Newton's method from the classical cosine estimates; the weights are
   2 / ((1 - x^2) P_n'(x)^2).  Nodes are returned in ascending order. */
void or_gauss_legendre(int n, double *x, double *w) {
  for (int i = 0; i < n; ++i) {
    double xi = -cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p = or_legendre(n, xi);
      double dp = or_legendre_deriv(n, 1, xi);
      double dx = p / dp;
      xi -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    double dp = or_legendre_deriv(n, 1, xi);
    x[i] = xi;
    w[i] = 2.0 / ((1.0 - xi * xi) * dp * dp);
  }
}

/* ---------------------------------------------------------------------------
 * Eq. (8): the weights c^l of the AT flux (7) over the q levels
 * l = k, k+1, ..., k+q-1 satisfy
 *     sum_l c^l (-l dt)^z / z! = 1 (z = 0), 0 (0 < z < q).
 * Multiplying row z by z!/dt^z gives the Vandermonde system
 *     sum_l c^l (-l)^z = delta_{z0},
 * solved here by Gauss-Jordan elimination in exact rational arithmetic
 * (64-bit numerator / denominator, reduced after every operation).
 * ------------------------------------------------------------------------- */
typedef struct { int64_t n, d; } frac;

static int64_t gcd64(int64_t a, int64_t b) {
  if (a < 0) a = -a;
  if (b < 0) b = -b;
  while (b) { int64_t t = a % b; a = b; b = t; }
  return a ? a : 1;
}
static frac fr(int64_t n, int64_t d) {
  if (d < 0) { n = -n; d = -d; }
  int64_t g = gcd64(n, d);
  frac r = {n / g, d / g};
  return r;
}
static frac q_sub(frac a, frac b) { return fr(a.n * b.d - b.n * a.d, a.d * b.d); }
static frac q_mul(frac a, frac b) { return fr(a.n * b.n, a.d * b.d); }
static frac q_div(frac a, frac b) { return fr(a.n * b.d, a.d * b.n); }

int or_at_coeffs(int q, int k, double *c) {
  if (q < 1 || q > 8 || k < 0) return -1;
  frac A[8][9];
  for (int z = 0; z < q; ++z) {
    for (int l = 0; l < q; ++l) {
      int64_t p = 1;
      for (int t = 0; t < z; ++t) p *= -(int64_t)(k + l);
      A[z][l] = fr(p, 1);
    }
    A[z][q] = fr(z == 0 ? 1 : 0, 1);
  }
  for (int col = 0; col < q; ++col) {
    int piv = -1;
    for (int r = col; r < q; ++r)
      if (A[r][col].n != 0) { piv = r; break; }
    if (piv < 0) return -2;
    if (piv != col)
      for (int t = 0; t <= q; ++t) { frac tmp = A[col][t]; A[col][t] = A[piv][t]; A[piv][t] = tmp; }
    frac p = A[col][col];
    for (int t = 0; t <= q; ++t) A[col][t] = q_div(A[col][t], p);
    for (int r = 0; r < q; ++r) {
      if (r == col || A[r][col].n == 0) continue;
      frac f = A[r][col];
      for (int t = 0; t <= q; ++t) A[r][t] = q_sub(A[r][t], q_mul(f, A[col][t]));
    }
  }
  for (int l = 0; l < q; ++l) c[l] = (double)A[l][q].n / (double)A[l][q].d;
  return 0;
}

/* ---------------------------------------------------------------------------
 * Buffer-element DoFs of Eq. (11), temporal and hybrid (spatio-temporal).
 *
 * Sec. 3.3 closes by noting that the temporal stencil of the buffer element
 * can be generalised to one that also uses delayed values at the element's
 * other nodes, with fewer buffered time levels for the same order.  Reading:
 * the Legendre coefficient j of a smooth field over an element of width dx
 * carries the factor dx^j (only derivatives of order >= j contribute to it),
 * and so do its time derivatives.  Extrapolating it in time from q_j levels
 * with the weights of Eq. (8) for q_j levels leaves an error of order
 * dt^{q_j} dx^j = dx^{r q_j + j} (dt ~ dx^r), so the order N_p + 1 of the
 * full temporal stencil needs only q_j = ceil((N_p + 1 - j)/r) levels for
 * mode j; for r = 1 and q levels in all, q_j = max(1, q - j).  In the values
 * at the element's nodes this is a stencil over (node, level): each node's
 * level-n value combines delayed values at all the element's nodes, and older
 * levels contribute only the element's low modes (the oldest one its mean).
 * ------------------------------------------------------------------------- */
int or_at_buffer(int q, int k, int V, int M, int hybrid, const double *levels, double *out) {
  if (q < 1 || q > 8 || k < 0 || V < 1 || M < 1) return -1;
  double c[8];
  for (int j = 0; j < M; ++j) {
    int qj = hybrid ? (q - j > 1 ? q - j : 1) : q;
    if (or_at_coeffs(qj, k, c)) return -1;
    for (int v = 0; v < V; ++v) {
      double acc = 0.0;
      for (int l = 0; l < qj; ++l) acc += c[l] * levels[((size_t)l * V + v) * M + j];
      out[v * M + j] = acc;
    }
  }
  return 0;
}

/* ---------------------------------------------------------------------------
 * Delay models, Sec. 4.
 * ------------------------------------------------------------------------- */

/* SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014): one step of
   the Weyl sequence followed by the variant-13 finaliser. */
uint64_t or_splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* The uniform number drawn for PE interface i at time step n (SAA, Sec. 4.2):
   a counter-based draw, so every interface and step has its own independent
   number no matter in which order they are evaluated.  53-bit mantissa in [0,1). */
double or_saa_uniform(uint64_t seed, int64_t n, int32_t i, int32_t n_if) {
  uint64_t ctr = (uint64_t)n * (uint64_t)n_if + (uint64_t)i;
  uint64_t z = or_splitmix64(seed ^ (ctr * 0x9E3779B97F4A7C15ull));
  return (double)(z >> 11) * 0x1.0p-53;
}

static int at_q(const or_config *cfg) {
  return cfg->at_order > 0 ? cfg->at_order : cfg->order_p + 1;
}

/* Delay drawn by the chosen model, before the start-up clamp.
 *   SYNC:     k = 0 (the synchronous algorithm).
 *   CAA:      k grows by one level per step and is reset when n % L == 0, i.e.
 *             k = n mod L at every interface (Sec. 4.1).
 *   SAA:      [0,1) is cut into L successive bins of widths p_0 .. p_{L-1}; the
 *             bin that holds the drawn number is the delay (Sec. 4.2).  Bins
 *             are closed on the left.
 *   SCHEDULE: an explicit table (tests), repeated with period schedule_steps. */
int or_raw_delay(const or_config *cfg, int32_t n_if, int64_t n, int32_t i) {
  switch (cfg->mode) {
    case OR_SYNC: return 0;
    case OR_CAA: return (int)(n % cfg->L);
    case OR_SAA: {
      double u = or_saa_uniform(cfg->seed, n, i, n_if);
      double cum = 0.0;
      for (int k = 0; k < cfg->L; ++k) {
        cum += cfg->pmf[k];
        if (u < cum) return k;
      }
      return cfg->L - 1;
    }
    case OR_SCHEDULE: {
      int64_t row = n % cfg->schedule_steps;
      return cfg->schedule[row * n_if + i];
    }
  }
  return 0;
}

/* Delay actually used at step n.  Levels before n = 0 do not exist, so a delay
   is clamped to k <= n - q + 1 (all q levels n-k .. n-k-q+1 exist); at the
   first steps the flux is synchronous. */
int or_eff_delay(const or_config *cfg, int32_t n_if, int64_t n, int32_t i) {
  int k = or_raw_delay(cfg, n_if, n, i);
  if (k <= 0) return 0;
  int64_t lim = n - at_q(cfg) + 1;
  if (lim < 0) lim = 0;
  if (k > lim) k = (int)lim;
  return k;
}

/* Dense Gauss-Jordan solve with partial pivoting; A is n x n row-major, b is
   n x nrhs row-major.  Solution returned in b. */
int or_dense_solve(int n, double *A, double *b, int nrhs) {
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(A[r * n + col]) > fabs(A[piv * n + col])) piv = r;
    if (A[piv * n + col] == 0.0) return -1;
    if (piv != col) {
      for (int t = 0; t < n; ++t) { double x = A[col * n + t]; A[col * n + t] = A[piv * n + t]; A[piv * n + t] = x; }
      for (int t = 0; t < nrhs; ++t) { double x = b[col * nrhs + t]; b[col * nrhs + t] = b[piv * nrhs + t]; b[piv * nrhs + t] = x; }
    }
    double p = A[col * n + col];
    for (int t = 0; t < n; ++t) A[col * n + t] /= p;
    for (int t = 0; t < nrhs; ++t) b[col * nrhs + t] /= p;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double f = A[r * n + col];
      if (f == 0.0) continue;
      for (int t = 0; t < n; ++t) A[r * n + t] -= f * A[col * n + t];
      for (int t = 0; t < nrhs; ++t) b[r * nrhs + t] -= f * b[col * nrhs + t];
    }
  }
  return 0;
}
