/*
 * ADG oracle — test infrastructure only.
 *
 * The ADG time step, in the order of the paper:
 *   Sec. 3.1  semi-discrete DG form Eq. (5) with the mass and stiffness matrices
 *             of Eq. (6) and the LDG auxiliary variable q = dw/dx (central trace
 *             for w, central diffusive flux)
 *   Sec. 3.2  at PE interfaces the numerical flux is the AT flux of Eq. (7): a
 *             combination of the single-valued synchronous fluxes of the levels
 *             n-k .. n-k-q+1, with the weights of Eq. (8)
 *   Sec. 3.3  after every Runge-Kutta stage the limiter; across PE interfaces the
 *             neighbour's modal data is the AT combination of Eq. (11)
 *   Sec. 4    emulated PEs, delays by CAA / SAA
 * Time integration is the three-stage SSP Runge-Kutta method of Shu & Osher.
 *
 * Readings (the paper is silent or ambiguous):
 *   * quadrature: Gauss-Legendre with N_p + 1 points unless n_quad is given; the
 *     volume term is quadrature of the nonlinear f(w_h) against phi'_i, and the
 *     source term of Eq. (5) is the L2 projection of s(w_h) (outside the 2/dx).
 *   * one delay k per PE interface per time step, shared by all stages and the
 *     limiter of that step; stage s of step n combines stage-s data of the levels
 *     n-k-j (the level spacing is dt for every stage).
 *   * the history at a PE interface holds, per level and stage: the synchronous
 *     flux (both sides at that level, with the synchronous central trace in the
 *     LDG gradient), the synchronous central trace of w (LDG), and both adjacent
 *     elements' unlimited stage outputs (for Eq. (11)).
 *   * a delay is clamped to k <= n - q + 1 so only existing levels are used; with
 *     k = 0 the synchronous value is used directly.
 *   * the periodic wrap face is a PE interface; transmissive faces are
 *     synchronous with the ghost trace equal to the interior trace.
 *
 * Pins (tests/test_oracle_solver.py): zero delays reproduce the synchronous
 * algorithm bit for bit; design order on the exact entropy wave with and without
 * delays; first order with the plain delayed flux; error growth with the number
 * of PEs; conservation of mass, momentum, energy and elements on periodic
 * domains under any delay pattern; sum_i rho Y_i = rho; Rankine-Hugoniot shock
 * speed; 0-D reactor against an ODE integration.  The troubled-cell indicator
 * (or_indicator; tests/test_oracle_limiter.py): KXRCF on constructed cells whose
 * indicator value is 0.9 or 1.1 at the inflow face, for both flow directions and
 * N_p = 1..3, with a larger jump at the outflow face (pins the threshold, the
 * exponent (N_p+1)/2 of h, the inflow face and the normaliser max_q |w(xi_q)|).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "or_internal.h"



struct or_solver {
  or_config cfg;
  /* owned copies of the configuration arrays */
  double *W, *nasa7, *A, *b, *Ea, *pmf;
  int32_t *nu_f, *nu_r, *pe_off;
  int8_t *schedule;

  int E, M, Q, V, ns, nif, q, nfaces;
  double dx, kx_h;                 /* element size, h^((Np+1)/2) of KXRCF */
  double xq[OR_MAXQ], wq[OR_MAXQ];
  double Bq[OR_MAXQ][OR_MAXM];     /* P_j(xi_q) */
  double Gq[OR_MAXQ][OR_MAXM];     /* P_j'(xi_q) */
  double Pm[OR_MAXM], Pp[OR_MAXM]; /* P_j(-1), P_j(+1) */
  double Minv[OR_MAXM * OR_MAXM];  /* inverse of the mass matrix of Eq. (6) */
  int *face_if, *if_face;

  double *w, *w1, *w2, *w3, *wu, *rhs;
  int S;                           /* stages per time step */
  double *kreg;                    /* 2N-storage register */
  double *tr_m, *tr_p;             /* traces at xi = -1, +1: [E][V] */
  double *fl;                      /* numerical flux per face [nfaces][V] */
  double *wc_sync, *wc_at;         /* central traces per face (LDG) */
  double *q_sync, *q_at;           /* LDG gradients [E][V][M] */
  int *kif;                        /* delay per interface for the current step */
  double *cif;                     /* AT weights per interface [nif][q] */

  int64_t n;
  int32_t max_steps;
  double *hF, *hWc, *hU;
  int8_t *flags;
  int64_t nflag_total;
  char msg[256];
};

#define IDX(e, v, j) (((size_t)(e) * s->V + (v)) * s->M + (j))

static int left_elem(const or_solver *s, int f) {
  if (s->cfg.bc == OR_PERIODIC) return (f - 1 + s->E) % s->E;
  return f - 1;             /* -1 at the left boundary */
}
static int right_elem(const or_solver *s, int f) {
  if (s->cfg.bc == OR_PERIODIC) return f % s->E;
  return f < s->E ? f : -1; /* -1 at the right boundary */
}
static int left_face(const or_solver *s, int e) { (void)s; return e; }
static int right_face(const or_solver *s, int e) {
  return s->cfg.bc == OR_PERIODIC ? (e + 1) % s->E : e + 1;
}

static double *hist_F(or_solver *s, int64_t m, int st, int i) {
  return s->hF + (((size_t)m * s->S + st) * s->nif + i) * s->V;
}
static double *hist_Wc(or_solver *s, int64_t m, int st, int i) {
  return s->hWc + (((size_t)m * s->S + st) * s->nif + i) * s->V;
}
static double *hist_U(or_solver *s, int64_t m, int st, int i, int side) {
  return s->hU + ((((size_t)m * s->S + st) * s->nif + i) * 2 + side) * (size_t)s->V * s->M;
}

static int fail(or_solver *s, const char *m) {
  snprintf(s->msg, sizeof s->msg, "%s (step %lld)", m, (long long)s->n);
  return -1;
}

static void *dup(const void *p, size_t bytes) {
  if (!p || !bytes) return NULL;
  void *q = malloc(bytes);
  memcpy(q, p, bytes);
  return q;
}

void or_destroy(or_solver *s) {
  if (!s) return;
  void *ptrs[] = {s->W, s->nasa7, s->A, s->b, s->Ea, s->pmf, s->nu_f, s->nu_r, s->pe_off, s->schedule,
                  s->face_if, s->if_face, s->w, s->w1, s->w2, s->w3, s->wu, s->rhs, s->tr_m, s->tr_p,
                  s->fl, s->wc_sync, s->wc_at, s->q_sync, s->q_at, s->kif, s->cif, s->hF, s->hWc,
                  s->hU, s->flags, s->kreg};
  for (size_t i = 0; i < sizeof ptrs / sizeof ptrs[0]; ++i) free(ptrs[i]);
  free(s);
}

int or_create(const or_config *cfg, const double *w0, int32_t max_steps, or_solver **out) {
  *out = NULL;
  if (cfg->n_species < 1 || cfg->n_species > OR_MAXNS) return -1;
  if (cfg->order_p < 0 || cfg->order_p + 1 > OR_MAXM) return -1;
  if (cfg->n_elem < 1 || cfg->n_pe < 1 || cfg->n_pe > cfg->n_elem) return -1;
  if (cfg->model == OR_ONESTEP && cfg->n_species != 2) return -1;
  if (cfg->limiter && cfg->model != OR_ONESTEP) return -1;
  if (cfg->mode != OR_SYNC && cfg->L < 1) return -1;
  if (cfg->at_stencil != OR_AT_TEMPORAL && cfg->at_stencil != OR_AT_HYBRID) return -1;
  if (cfg->limiter && (cfg->indicator < OR_KXRCF || cfg->indicator > OR_ALL)) return -1;
  or_solver *s = calloc(1, sizeof *s);
  s->cfg = *cfg;
  int ns = cfg->n_species, nr = cfg->n_reactions;
  if (cfg->model == OR_DETAILED) {
    s->W = dup(cfg->W, sizeof(double) * ns);
    s->nasa7 = dup(cfg->nasa7, sizeof(double) * 7 * ns);
    s->A = dup(cfg->A, sizeof(double) * nr);
    s->b = dup(cfg->b, sizeof(double) * nr);
    s->Ea = dup(cfg->Ea, sizeof(double) * nr);
    s->nu_f = dup(cfg->nu_f, sizeof(int32_t) * nr * ns);
    s->nu_r = dup(cfg->nu_r, sizeof(int32_t) * nr * ns);
    s->cfg.W = s->W; s->cfg.nasa7 = s->nasa7; s->cfg.A = s->A; s->cfg.b = s->b; s->cfg.Ea = s->Ea;
    s->cfg.nu_f = s->nu_f; s->cfg.nu_r = s->nu_r;
  }
  if (cfg->mode == OR_SAA) {
    s->pmf = dup(cfg->pmf, sizeof(double) * cfg->L);
    s->cfg.pmf = s->pmf;
  }
  s->E = cfg->n_elem;
  s->M = cfg->order_p + 1;
  s->Q = cfg->n_quad > 0 ? cfg->n_quad : s->M;
  if (s->Q > OR_MAXQ) { or_destroy(s); return -1; }
  s->V = 3 + ns;
  s->ns = ns;
  s->q = cfg->at_order > 0 ? cfg->at_order : cfg->order_p + 1;
  s->nfaces = cfg->bc == OR_PERIODIC ? s->E : s->E + 1;
  s->nif = cfg->bc == OR_PERIODIC ? cfg->n_pe : cfg->n_pe - 1;
  if (cfg->mode == OR_SCHEDULE) {
    if (cfg->schedule_steps < 1) { or_destroy(s); return -1; }
    s->schedule = dup(cfg->schedule, (size_t)cfg->schedule_steps * (s->nif > 0 ? s->nif : 1));
    s->cfg.schedule = s->schedule;
    /* a schedule holds delays from the L admissible ones, 0..L-1 (Sec. 4) */
    for (size_t t = 0; t < (size_t)cfg->schedule_steps * (size_t)s->nif; ++t)
      if (s->schedule[t] < 0 || s->schedule[t] >= cfg->L) { or_destroy(s); return -1; }
  }
  s->pe_off = malloc(sizeof(int32_t) * (cfg->n_pe + 1));
  for (int p = 0; p <= cfg->n_pe; ++p)
    s->pe_off[p] = cfg->pe_offsets ? cfg->pe_offsets[p] : (int32_t)(((int64_t)p * s->E) / cfg->n_pe);
  s->cfg.pe_offsets = s->pe_off;
  for (int p = 0; p < cfg->n_pe; ++p)
    if (s->pe_off[p + 1] <= s->pe_off[p]) { or_destroy(s); return -1; }
  if (s->pe_off[0] != 0 || s->pe_off[cfg->n_pe] != s->E) { or_destroy(s); return -1; }

  s->dx = (cfg->x_right - cfg->x_left) / s->E;
  s->kx_h = pow(s->dx, 0.5 * (cfg->order_p + 1));
  or_gauss_legendre(s->Q, s->xq, s->wq);
  for (int q = 0; q < s->Q; ++q)
    for (int j = 0; j < s->M; ++j) {
      s->Bq[q][j] = or_legendre(j, s->xq[q]);
      s->Gq[q][j] = or_legendre_deriv(j, 1, s->xq[q]);
    }
  for (int j = 0; j < s->M; ++j) {
    s->Pm[j] = or_legendre(j, -1.0);
    s->Pp[j] = or_legendre(j, 1.0);
  }
  /* Eq. (6): M_ij = int phi_j phi_i dxi by quadrature, then its inverse. */
  {
    int M = s->M;
    double Mm[OR_MAXM * OR_MAXM];
    double xg[OR_MAXQ], wg[OR_MAXQ];
    or_gauss_legendre(M, xg, wg);
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) {
        double acc = 0.0;
        for (int q = 0; q < M; ++q) acc += wg[q] * or_legendre(j, xg[q]) * or_legendre(i, xg[q]);
        Mm[i * M + j] = acc;
        s->Minv[i * M + j] = i == j ? 1.0 : 0.0;
      }
    if (or_dense_solve(M, Mm, s->Minv, M)) { or_destroy(s); return -1; }
  }
  s->face_if = malloc(sizeof(int) * (s->nfaces + 1));
  for (int f = 0; f <= s->nfaces; ++f) s->face_if[f] = -1;
  s->if_face = malloc(sizeof(int) * (s->nif > 0 ? s->nif : 1));
  if (cfg->bc == OR_PERIODIC) {
    for (int p = 0; p < cfg->n_pe; ++p) { s->face_if[s->pe_off[p]] = p; s->if_face[p] = s->pe_off[p]; }
  } else {
    for (int p = 1; p < cfg->n_pe; ++p) { s->face_if[s->pe_off[p]] = p - 1; s->if_face[p - 1] = s->pe_off[p]; }
  }
  size_t nst = (size_t)s->E * s->V * s->M;
  s->w = malloc(sizeof(double) * nst);
  s->w1 = malloc(sizeof(double) * nst);
  s->w2 = malloc(sizeof(double) * nst);
  s->w3 = malloc(sizeof(double) * nst);
  if (cfg->rk < OR_SSPRK3 || cfg->rk > OR_LSERK4) { or_destroy(s); return -1; }
  s->S = cfg->rk == OR_SSPRK3 ? 3 : cfg->rk == OR_RK2 ? 2 : 5;
  s->kreg = calloc(nst, sizeof(double));
  s->wu = malloc(sizeof(double) * nst);
  s->rhs = malloc(sizeof(double) * nst);
  s->q_sync = calloc(nst, sizeof(double));
  s->q_at = calloc(nst, sizeof(double));
  s->tr_m = malloc(sizeof(double) * s->E * s->V);
  s->tr_p = malloc(sizeof(double) * s->E * s->V);
  s->fl = malloc(sizeof(double) * (s->nfaces + 1) * s->V);
  s->wc_sync = malloc(sizeof(double) * (s->nfaces + 1) * s->V);
  s->wc_at = malloc(sizeof(double) * (s->nfaces + 1) * s->V);
  s->kif = calloc(s->nif > 0 ? s->nif : 1, sizeof(int));
  s->cif = calloc((size_t)(s->nif > 0 ? s->nif : 1) * s->q, sizeof(double));
  s->flags = calloc(s->E, 1);
  memcpy(s->w, w0, sizeof(double) * nst);
  s->max_steps = max_steps;
  if (cfg->mode != OR_SYNC && s->nif > 0) {
    size_t lv = (size_t)max_steps * s->S * s->nif;
    s->hF = calloc(lv * s->V, sizeof(double));
    s->hWc = calloc(lv * s->V, sizeof(double));
    s->hU = calloc(lv * 2 * s->V * s->M, sizeof(double));
    if (!s->hF || !s->hWc || !s->hU) { or_destroy(s); return -2; }
  }
  s->n = 0;
  *out = s;
  return 0;
}

/* Modal -> point value of variable v of element e at a point with basis values P. */
static double eval_modes(const or_solver *s, const double *we, int v, const double *P) {
  double acc = 0.0;
  for (int j = 0; j < s->M; ++j) acc += we[v * s->M + j] * P[j];
  return acc;
}

/* LDG auxiliary variable of Sec. 3.1 in element e, from the central traces at
   its two faces: q = (2/dx) M^-1 ( w*_{e+1} phi(1) - w*_e phi(-1) - S w ),
   (S w)_i = int w phi_i' dxi by quadrature. */
static void ldg_gradient(const or_solver *s, const double *we, const double *wc_l, const double *wc_r, double *qe) {
  int M = s->M;
  for (int v = 0; v < s->V; ++v) {
    double bvec[OR_MAXM];
    for (int i = 0; i < M; ++i) bvec[i] = wc_r[v] * s->Pp[i] - wc_l[v] * s->Pm[i];
    for (int q = 0; q < s->Q; ++q) {
      double wqv = eval_modes(s, we, v, s->Bq[q]);
      for (int i = 0; i < M; ++i) bvec[i] -= s->wq[q] * s->Gq[q][i] * wqv;
    }
    for (int i = 0; i < M; ++i) {
      double acc = 0.0;
      for (int j = 0; j < M; ++j) acc += s->Minv[i * M + j] * bvec[j];
      qe[v * M + i] = 2.0 / s->dx * acc;
    }
  }
}

/* Trace of the modal field g of element e at xi = -1 (side 0) or +1 (side 1). */
static void trace_of(const or_solver *s, const double *ge, int side, double *out) {
  for (int v = 0; v < s->V; ++v) out[v] = eval_modes(s, ge, v, side ? s->Pp : s->Pm);
}

/* Full numerical flux at a face from its two traces and (LDG) their gradients:
   f_hat = f_hat^c(w-, w+) - (f^d(w-, q-) + f^d(w+, q+)) / 2. */
static int face_flux(or_solver *s, const double *wL, const double *wR, const double *qL, const double *qR, double *f) {
  if (or_num_flux(&s->cfg, wL, wR, f)) return -1;
  if (s->cfg.model == OR_DETAILED && s->cfg.viscous) {
    double fdL[OR_MAXV], fdR[OR_MAXV];
    if (or_diff_flux(&s->cfg, wL, qL, fdL) || or_diff_flux(&s->cfg, wR, qR, fdR)) return -1;
    for (int v = 0; v < s->V; ++v) f[v] -= 0.5 * (fdL[v] + fdR[v]);
  }
  return 0;
}

/* The AT combination of Eq. (7)/(11) over q past levels of a history record.  The
   buffer-element DoFs (which = 2) follow the temporal or the hybrid stencil (or_at_buffer). */
static void at_combine(or_solver *s, int i, int st, int which, int side, int len, double *out) {
  int k = s->kif[i];
  if (which == 2) {
    double lv[8 * OR_MAXV * OR_MAXM];
    for (int j = 0; j < s->q; ++j)
      memcpy(lv + (size_t)j * len, hist_U(s, s->n - k - j, st, i, side), sizeof(double) * len);
    or_at_buffer(s->q, k, s->V, s->M, s->cfg.at_stencil == OR_AT_HYBRID, lv, out);
    return;
  }
  for (int t = 0; t < len; ++t) out[t] = 0.0;
  for (int j = 0; j < s->q; ++j) {
    int64_t m = s->n - k - j;
    const double *h = which == 0 ? hist_F(s, m, st, i) : hist_Wc(s, m, st, i);
    for (int t = 0; t < len; ++t) out[t] += s->cif[i * s->q + j] * h[t];
  }
}

/* Right-hand side of Eq. (5) for every element at stage st of step n. */
static int compute_rhs(or_solver *s, int st, const double *w, double *rhs) {
  int E = s->E, V = s->V, M = s->M;
  int visc = s->cfg.model == OR_DETAILED && s->cfg.viscous;
  int keep_hist = s->hF != NULL;
  for (int e = 0; e < E; ++e) {
    trace_of(s, w + IDX(e, 0, 0), 0, s->tr_m + (size_t)e * V);
    trace_of(s, w + IDX(e, 0, 0), 1, s->tr_p + (size_t)e * V);
  }
  /* traces on both sides of every face; ghost = interior at physical boundaries */
#define TRACE_L(f) (left_elem(s, f) >= 0 ? s->tr_p + (size_t)left_elem(s, f) * V : s->tr_m + (size_t)right_elem(s, f) * V)
#define TRACE_R(f) (right_elem(s, f) >= 0 ? s->tr_m + (size_t)right_elem(s, f) * V : s->tr_p + (size_t)left_elem(s, f) * V)

  if (visc) {
    for (int f = 0; f < s->nfaces; ++f) {
      const double *wL = TRACE_L(f), *wR = TRACE_R(f);
      double *c = s->wc_sync + (size_t)f * V, *ca = s->wc_at + (size_t)f * V;
      for (int v = 0; v < V; ++v) c[v] = 0.5 * (wL[v] + wR[v]);
      int i = s->face_if[f];
      if (i >= 0 && keep_hist) {
        memcpy(hist_Wc(s, s->n, st, i), c, sizeof(double) * V);
        if (s->kif[i] > 0) { at_combine(s, i, st, 1, 0, V, ca); continue; }
      }
      memcpy(ca, c, sizeof(double) * V);
    }
    for (int e = 0; e < E; ++e) {
      int lf = left_face(s, e), rf = right_face(s, e);
      ldg_gradient(s, w + IDX(e, 0, 0), s->wc_sync + (size_t)lf * V, s->wc_sync + (size_t)rf * V, s->q_sync + IDX(e, 0, 0));
      ldg_gradient(s, w + IDX(e, 0, 0), s->wc_at + (size_t)lf * V, s->wc_at + (size_t)rf * V, s->q_at + IDX(e, 0, 0));
    }
  }

  for (int f = 0; f < s->nfaces; ++f) {
    int le = left_elem(s, f), re = right_elem(s, f);
    const double *wL = TRACE_L(f), *wR = TRACE_R(f);
    double *F = s->fl + (size_t)f * V;
    int i = s->face_if[f];
    /* gradient traces at the face: synchronous ones for the PE-interface record,
       the ones the adjacent elements actually hold otherwise */
    double qLs[OR_MAXV] = {0}, qRs[OR_MAXV] = {0}, qLa[OR_MAXV] = {0}, qRa[OR_MAXV] = {0};
    if (visc) {
      if (le >= 0) { trace_of(s, s->q_sync + IDX(le, 0, 0), 1, qLs); trace_of(s, s->q_at + IDX(le, 0, 0), 1, qLa); }
      if (re >= 0) { trace_of(s, s->q_sync + IDX(re, 0, 0), 0, qRs); trace_of(s, s->q_at + IDX(re, 0, 0), 0, qRa); }
      if (le < 0) { memcpy(qLs, qRs, sizeof qLs); memcpy(qLa, qRa, sizeof qLa); }
      if (re < 0) { memcpy(qRs, qLs, sizeof qRs); memcpy(qRa, qLa, sizeof qRa); }
    }
    if (i >= 0) {
      double Fs[OR_MAXV];
      if (face_flux(s, wL, wR, qLs, qRs, Fs)) return fail(s, "non-physical state at a PE interface");
      if (keep_hist) memcpy(hist_F(s, s->n, st, i), Fs, sizeof(double) * V);
      if (keep_hist && s->kif[i] > 0) at_combine(s, i, st, 0, 0, V, F);
      else memcpy(F, Fs, sizeof(double) * V);
    } else {
      if (face_flux(s, wL, wR, qLa, qRa, F)) return fail(s, "non-physical state at a face");
    }
  }
#undef TRACE_L
#undef TRACE_R

  for (int e = 0; e < E; ++e) {
    const double *we = w + IDX(e, 0, 0);
    double bvec[OR_MAXV][OR_MAXM], svec[OR_MAXV][OR_MAXM];
    memset(bvec, 0, sizeof bvec);
    memset(svec, 0, sizeof svec);
    for (int q = 0; q < s->Q; ++q) {
      double wqv[OR_MAXV], f[OR_MAXV], src[OR_MAXV];
      for (int v = 0; v < V; ++v) wqv[v] = eval_modes(s, we, v, s->Bq[q]);
      or_prim pr;
      if (or_primitives(&s->cfg, wqv, &pr)) return fail(s, "non-physical state at a quadrature node");
      or_flux_from_prim(&s->cfg, wqv, &pr, f);
      if (visc) {
        double dq[OR_MAXV], fd[OR_MAXV];
        for (int v = 0; v < V; ++v) dq[v] = eval_modes(s, s->q_at + IDX(e, 0, 0), v, s->Bq[q]);
        or_diff_flux_from_prim(&s->cfg, wqv, &pr, dq, fd);
        for (int v = 0; v < V; ++v) f[v] -= fd[v];
      }
      or_source_from_prim(&s->cfg, wqv, &pr, src);
      for (int v = 0; v < V; ++v)
        for (int i = 0; i < M; ++i) {
          bvec[v][i] += s->wq[q] * s->Gq[q][i] * f[v];
          svec[v][i] += s->wq[q] * s->Bq[q][i] * src[v];
        }
    }
    const double *Fl = s->fl + (size_t)left_face(s, e) * V, *Fr = s->fl + (size_t)right_face(s, e) * V;
    for (int v = 0; v < V; ++v)
      for (int i = 0; i < M; ++i) bvec[v][i] += -Fr[v] * s->Pp[i] + Fl[v] * s->Pm[i];
    for (int v = 0; v < V; ++v)
      for (int i = 0; i < M; ++i) {
        double a = 0.0, c = 0.0;
        for (int j = 0; j < M; ++j) {
          a += s->Minv[i * M + j] * bvec[v][j];
          c += s->Minv[i * M + j] * svec[v][j];
        }
        rhs[IDX(e, v, i)] = 2.0 / s->dx * a + c;
      }
  }
  return 0;
}

/* KXRCF indicator of element e, from its modal data and the traces of its two
   neighbours facing it; jumps are summed over inflow faces only. */
static int kxrcf_flag(or_solver *s, const double *we, const double *nbL_tr, const double *nbR_tr, int ghostL, int ghostR) {
  int V = s->V;
  double tm[OR_MAXV], tp[OR_MAXV];
  trace_of(s, we, 0, tm);
  trace_of(s, we, 1, tp);
  double uL_e = tm[1] / tm[0], uR_e = tp[1] / tp[0];
  double uL_n = ghostL ? uL_e : nbL_tr[1] / nbL_tr[0];
  double uR_n = ghostR ? uR_e : nbR_tr[1] / nbR_tr[0];
  int vars[2] = {0, 2};
  int flag = 0;
  for (int t = 0; t < 2; ++t) {
    int v = vars[t];
    double jump = 0.0;
    if (0.5 * (uL_e + uL_n) > 0.0 && !ghostL) jump += tm[v] - nbL_tr[v];
    if (0.5 * (uR_e + uR_n) < 0.0 && !ghostR) jump += tp[v] - nbR_tr[v];
    double norm = 0.0;
    for (int q = 0; q < s->Q; ++q) {
      double val = fabs(eval_modes(s, we, v, s->Bq[q]));
      if (val > norm) norm = val;
    }
    if (fabs(jump) / (s->kx_h * norm) > 1.0) flag = 1;
  }
  (void)V;
  return flag;
}

/* minmod of three numbers: the one of least magnitude if all share a sign, else 0. */
static double minmod3(double a, double b, double c) {
  if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
  if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
  return 0.0;
}

/* TVB minmod troubled-cell test (the TVD slope-limiter indicator of Sec. 3.3 when
   M = 0), on every conserved variable.  With the cell mean a (mode 0), the face
   deviations d+ = w(+1) - a and d- = a - w(-1) and the mean differences
   D+ = a_{e+1} - a, D- = a - a_{e-1}: the cell is troubled when, for either face,
   the modified value (d itself if |d| <= M dx^2, else minmod(d, D+, D-)) differs
   from d by more than 1e-10 of the largest |mean| of any variable in the stencil
   (round-off in a constant state is not a slope; a variable that is zero there,
   such as the momentum of gas at rest, takes the scale of the others).
   Neighbours are the unlimited data (Eq. (11) at delayed PE faces); a ghost
   neighbour repeats the cell's own mean. */
static int minmod_flag(or_solver *s, const double *we, const double *nbL, const double *nbR) {
  int V = s->V, M = s->M;
  double mh2 = s->cfg.tvb_m * s->dx * s->dx;
  double tm[OR_MAXV], tp[OR_MAXV];
  trace_of(s, we, 0, tm);
  trace_of(s, we, 1, tp);
  double scale = 0.0;
  for (int v = 0; v < V; ++v)
    scale = fmax(scale, fmax(fabs(we[v * M]), fmax(fabs(nbL[v * M]), fabs(nbR[v * M]))));
  double tol = 1e-10 * scale;
  for (int v = 0; v < V; ++v) {
    double a = we[v * M], aL = nbL[v * M], aR = nbR[v * M];
    double dp = tp[v] - a, dm = a - tm[v], Dp = aR - a, Dm = a - aL;
    double mp = fabs(dp) <= mh2 ? dp : minmod3(dp, Dp, Dm);
    double mm = fabs(dm) <= mh2 ? dm : minmod3(dm, Dp, Dm);
    if (fabs(mp - dp) > tol || fabs(mm - dm) > tol) return 1;
  }
  return 0;
}

/* Limiter over the unlimited stage output wu -> wl (Jacobi: every stencil reads
   unlimited data; across a delayed PE interface the neighbour is Eq. (11)). */
static int apply_limiter(or_solver *s, int st, const double *wu, double *wl) {
  int E = s->E, V = s->V, M = s->M;
  size_t blk = (size_t)V * M;
  double nbL[OR_MAXV * OR_MAXM], nbR[OR_MAXV * OR_MAXM];
  for (int e = 0; e < E; ++e) {
    const double *we = wu + IDX(e, 0, 0);
    int lf = left_face(s, e), rf = right_face(s, e);
    int le = left_elem(s, lf), re = right_elem(s, rf);
    int ghostL = le < 0, ghostR = re < 0;
    int il = s->face_if[lf], ir = s->face_if[rf];
    if (ghostL) {
      memset(nbL, 0, sizeof nbL);
      for (int v = 0; v < V; ++v) nbL[v * M] = we[v * M];
    } else if (il >= 0 && s->hU && s->kif[il] > 0) {
      at_combine(s, il, st, 2, 0, (int)blk, nbL);
    } else {
      memcpy(nbL, wu + IDX(le, 0, 0), sizeof(double) * blk);
    }
    if (ghostR) {
      memset(nbR, 0, sizeof nbR);
      for (int v = 0; v < V; ++v) nbR[v * M] = we[v * M];
    } else if (ir >= 0 && s->hU && s->kif[ir] > 0) {
      at_combine(s, ir, st, 2, 1, (int)blk, nbR);
    } else {
      memcpy(nbR, wu + IDX(re, 0, 0), sizeof(double) * blk);
    }
    double trL[OR_MAXV], trR[OR_MAXV];
    trace_of(s, nbL, 1, trL);
    trace_of(s, nbR, 0, trR);
    int fl = s->cfg.indicator == OR_MINMOD ? minmod_flag(s, we, nbL, nbR)
             : s->cfg.indicator == OR_ALL  ? 1
                                           : kxrcf_flag(s, we, trL, trR, ghostL, ghostR);
    s->flags[e] = (int8_t)fl;
    if (fl) {
      s->nflag_total++;
      if (or_weno_cell(&s->cfg, nbL, we, nbR, wl + IDX(e, 0, 0))) return fail(s, "limiter failed");
    } else {
      memcpy(wl + IDX(e, 0, 0), we, sizeof(double) * blk);
    }
  }
  return 0;
}

/* 2N-storage low-storage Runge-Kutta schemes (Williamson's form): per stage
   k <- A_s k + dt L(u), u <- u + B_s k.
   RK2: A = (0, -1), B = (1, 1/2), which is Heun's two-stage second-order method
   (u1 = u + dt L(u), u^{n+1} = (u + u1 + dt L(u1))/2).
   LSERK4: the five-stage fourth-order scheme of Carpenter and Kennedy (NASA
   TM-109112, 1994), the usual "LSERK" of DG solvers. */
static const double kRK2A[2] = {0.0, -1.0};
static const double kRK2B[2] = {1.0, 0.5};
static const double kLSA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                               -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
static const double kLSB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                               1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                               2277821191437.0 / 14882151754819.0};

/* History record of the PE-interface elements of a stage output, then the
   limiter (which turns the unlimited output u into w_out). */
static int finish_stage(or_solver *s, int st, double *u, double *w_out) {
  if (s->hU) {
    for (int i = 0; i < s->nif; ++i) {
      int f = s->if_face[i];
      int le = left_elem(s, f), re = right_elem(s, f);
      memcpy(hist_U(s, s->n, st, i, 0), u + IDX(le, 0, 0), sizeof(double) * s->V * s->M);
      memcpy(hist_U(s, s->n, st, i, 1), u + IDX(re, 0, 0), sizeof(double) * s->V * s->M);
    }
  }
  if (s->cfg.limiter) return apply_limiter(s, st, u, w_out);
  return 0;
}

/* One SSP-RK3 stage (Shu-Osher form): w_out = a0 w_base + a1 (w_in + dt L(w_in)). */
static int do_stage(or_solver *s, int st, const double *w_in, const double *w_base, double *w_out) {
  size_t nst = (size_t)s->E * s->V * s->M;
  if (compute_rhs(s, st, w_in, s->rhs)) return -1;
  double dt = s->cfg.dt;
  double *dst = s->cfg.limiter ? s->wu : w_out;
  for (size_t t = 0; t < nst; ++t) {
    double y = w_in[t] + dt * s->rhs[t];
    if (st == 0) dst[t] = y;
    else if (st == 1) dst[t] = 0.75 * w_base[t] + 0.25 * y;
    else dst[t] = (1.0 / 3.0) * w_base[t] + (2.0 / 3.0) * y;
  }
  return finish_stage(s, st, dst, w_out);
}

/* One stage of a 2N-storage scheme: k = A k + dt L(u_in); u_out = u_in + B k. */
static int do_stage_2n(or_solver *s, int st, double A, double B, const double *u_in, double *u_out) {
  size_t nst = (size_t)s->E * s->V * s->M;
  if (compute_rhs(s, st, u_in, s->rhs)) return -1;
  double dt = s->cfg.dt;
  double *dst = s->cfg.limiter ? s->wu : u_out;
  for (size_t t = 0; t < nst; ++t) {
    s->kreg[t] = A * s->kreg[t] + dt * s->rhs[t];
    dst[t] = u_in[t] + B * s->kreg[t];
  }
  return finish_stage(s, st, dst, u_out);
}

int or_step(or_solver *s, int32_t n_steps) {
  size_t nst = (size_t)s->E * s->V * s->M;
  for (int32_t t = 0; t < n_steps; ++t) {
    if (s->hF && s->n >= s->max_steps) return fail(s, "history exhausted (max_steps)");
    for (int i = 0; i < s->nif; ++i) {
      s->kif[i] = or_eff_delay(&s->cfg, s->nif, s->n, i);
      if (or_at_coeffs(s->q, s->kif[i], s->cif + (size_t)i * s->q)) return fail(s, "AT weights");
    }
    if (s->cfg.rk == OR_SSPRK3) {
      if (do_stage(s, 0, s->w, s->w, s->w1)) return -1;
      if (do_stage(s, 1, s->w1, s->w, s->w2)) return -1;
      if (do_stage(s, 2, s->w2, s->w, s->w3)) return -1;
      memcpy(s->w, s->w3, sizeof(double) * nst);
    } else {
      const double *A = s->cfg.rk == OR_RK2 ? kRK2A : kLSA;
      const double *B = s->cfg.rk == OR_RK2 ? kRK2B : kLSB;
      double *u = s->w, *v = s->w1;
      for (int st = 0; st < s->S; ++st) {
        if (do_stage_2n(s, st, A[st], B[st], u, v)) return -1;
        double *x = u; u = v; v = x;
      }
      if (u != s->w) memcpy(s->w, u, sizeof(double) * nst);
    }
    s->n++;
  }
  return 0;
}

int or_get_state(const or_solver *s, double *w) {
  memcpy(w, s->w, sizeof(double) * (size_t)s->E * s->V * s->M);
  return 0;
}
int64_t or_get_step(const or_solver *s) { return s->n; }
int or_get_flags(const or_solver *s, int8_t *flags) {
  memcpy(flags, s->flags, s->E);
  return 0;
}
int64_t or_total_flags(const or_solver *s) { return s->nflag_total; }
const char *or_error(const or_solver *s) { return s->msg; }
int32_t or_n_interfaces(const or_solver *s) { return s->nif; }

/* Synchronous right-hand side of Eq. (5) for a state (no delays, step 0). */
int or_rhs_sync(const or_config *cfg, const double *w, double *rhs) {
  or_config c = *cfg;
  c.mode = OR_SYNC;
  or_solver *s;
  if (or_create(&c, w, 1, &s)) return -1;
  int rc = compute_rhs(s, 0, s->w, rhs);
  or_destroy(s);
  return rc;
}

/* Troubled-cell indicator of Sec. 3.3 for one cell with modal data we and
   neighbours nbL, nbR ([V][M] each; a ghost neighbour is ignored by KXRCF and
   taken as the cell's own mean by the minmod test, as in the limiter). */
int or_indicator(const or_config *cfg, const double *nbL, const double *we, const double *nbR, int ghostL,
                 int ghostR) {
  or_config c = *cfg;
  c.mode = OR_SYNC;
  size_t nst = (size_t)cfg->n_elem * (3 + cfg->n_species) * (cfg->order_p + 1);
  double *w0 = calloc(nst, sizeof(double));
  or_solver *s;
  int rc = or_create(&c, w0, 1, &s);
  free(w0);
  if (rc) return -1;
  int V = s->V, M = s->M;
  double gL[OR_MAXV * OR_MAXM], gR[OR_MAXV * OR_MAXM];
  memcpy(gL, nbL, sizeof(double) * V * M);
  memcpy(gR, nbR, sizeof(double) * V * M);
  if (ghostL) { memset(gL, 0, sizeof gL); for (int v = 0; v < V; ++v) gL[v * M] = we[v * M]; }
  if (ghostR) { memset(gR, 0, sizeof gR); for (int v = 0; v < V; ++v) gR[v * M] = we[v * M]; }
  double trL[OR_MAXV], trR[OR_MAXV];
  trace_of(s, gL, 1, trL);
  trace_of(s, gR, 0, trR);
  int fl = s->cfg.indicator == OR_MINMOD ? minmod_flag(s, we, gL, gR)
           : s->cfg.indicator == OR_ALL  ? 1
                                         : kxrcf_flag(s, we, trL, trR, ghostL, ghostR);
  or_destroy(s);
  return fl;
}

/* LDG gradient q of Sec. 3.1 with synchronous central traces. */
int or_gradient_sync(const or_config *cfg, const double *w, double *qout) {
  or_config c = *cfg;
  c.mode = OR_SYNC;
  or_solver *s;
  if (or_create(&c, w, 1, &s)) return -1;
  int V = s->V;
  for (int e = 0; e < s->E; ++e) {
    trace_of(s, w + IDX(e, 0, 0), 0, s->tr_m + (size_t)e * V);
    trace_of(s, w + IDX(e, 0, 0), 1, s->tr_p + (size_t)e * V);
  }
  for (int f = 0; f < s->nfaces; ++f) {
    int le = left_elem(s, f), re = right_elem(s, f);
    const double *wL = le >= 0 ? s->tr_p + (size_t)le * V : s->tr_m + (size_t)re * V;
    const double *wR = re >= 0 ? s->tr_m + (size_t)re * V : s->tr_p + (size_t)le * V;
    for (int v = 0; v < V; ++v) s->wc_sync[(size_t)f * V + v] = 0.5 * (wL[v] + wR[v]);
  }
  for (int e = 0; e < s->E; ++e)
    ldg_gradient(s, w + IDX(e, 0, 0), s->wc_sync + (size_t)left_face(s, e) * V,
                 s->wc_sync + (size_t)right_face(s, e) * V, qout + IDX(e, 0, 0));
  or_destroy(s);
  return 0;
}
