/*
 * ADG oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar-loop FP64 CPU implementation of the asynchronous
 * discontinuous Galerkin (ADG) solver of Arumugam & Aditya, "An asynchronous
 * discontinuous Galerkin method for combustion simulations" (arXiv 2501.01747).
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or constant with the HIP library:
 * everything below is written from the paper, Sec. 2-4.
 *
 * State layout used everywhere in the oracle: w[e][v][j], element e, conserved
 * variable v (rho, rho u, rho E, rho Y_1 .. rho Y_Ns; Eq. (2)), Legendre mode j.
 *
 * Parity status per function is listed in the header of each source file.
 */
#ifndef ADG_ORACLE_H
#define ADG_ORACLE_H

#include <stdint.h>

enum { OR_ONESTEP = 0, OR_DETAILED = 1 };
enum { OR_PERIODIC = 0, OR_TRANSMISSIVE = 1 };
enum { OR_RUSANOV = 0, OR_HLLC = 1 };
enum { OR_SYNC = 0, OR_CAA = 1, OR_SAA = 2, OR_SCHEDULE = 3 };
enum { OR_KXRCF = 0, OR_MINMOD = 1, OR_ALL = 2 };
enum { OR_AT_TEMPORAL = 0, OR_AT_HYBRID = 1 };
enum { OR_SSPRK3 = 0, OR_RK2 = 1, OR_LSERK4 = 2 };

typedef struct {
  /* ---- physics, Sec. 2 ---- */
  int32_t model;          /* OR_ONESTEP: reactive Euler, one irreversible step R -> P
                             OR_DETAILED: reversible mass-action mechanism, NASA-7 thermo */
  int32_t n_species;      /* N_s; number of conserved variables V = 3 + N_s */
  int32_t viscous;        /* detailed model only: 1 = Navier-Stokes terms of Eq. (2)-(3) via LDG */
  double gamma, q_heat, e_act, k_pre;  /* one-step model (nondimensional, R = 1) */
  int32_t n_reactions;
  const double *W;        /* [Ns] kg/mol */
  const double *nasa7;    /* [Ns][7] single temperature range */
  const int32_t *nu_f;    /* [Nr][Ns] reactant stoichiometric coefficients */
  const int32_t *nu_r;    /* [Nr][Ns] product stoichiometric coefficients */
  const double *A, *b, *Ea; /* [Nr] k_f = A T^b exp(-Ea/(Ru T)), SI */
  double Ru, p_ref;       /* gas constant J/(mol K) and standard pressure Pa */
  double mu_ref, T_ref, mu_exp, prandtl;  /* mu = mu_ref (T/T_ref)^mu_exp, k = mu cp/Pr, Le = 1 */
  double T_guess;         /* fixed Newton start for T(e) */
  /* ---- discretisation, Sec. 3.1 ---- */
  int32_t order_p;        /* N_p */
  int32_t n_quad;         /* Gauss-Legendre points per element (0 = N_p + 1) */
  int32_t n_elem;
  double x_left, x_right;
  int32_t bc;             /* OR_PERIODIC | OR_TRANSMISSIVE */
  int32_t flux;           /* OR_RUSANOV | OR_HLLC */
  int32_t limiter;        /* 1 = troubled-cell indicator + characteristic (AT-)WENO, Sec. 3.3 */
  int32_t indicator;      /* OR_KXRCF | OR_MINMOD (TVB minmod on the conserved variables) |
                             OR_ALL (every cell limited: the accuracy-test setting of the WENO limiter) */
  double tvb_m;           /* TVB constant M of the minmod test (0 = TVD) */
  double weno_gamma[3];   /* linear weights gamma_{-1}, gamma_0, gamma_{+1} */
  double weno_eps;
  double dt;
  int32_t rk;             /* OR_SSPRK3 (Shu-Osher) | OR_RK2 | OR_LSERK4 (2N-storage schemes) */
  /* ---- asynchrony, Sec. 3.2 and Sec. 4 ---- */
  int32_t n_pe;
  const int32_t *pe_offsets;   /* [n_pe + 1] element offsets, or NULL = floor(p E / P) */
  int32_t mode;           /* OR_SYNC | OR_CAA | OR_SAA | OR_SCHEDULE */
  int32_t L;              /* number of admissible delays: k in {0 .. L-1} */
  const double *pmf;      /* [L] SAA probabilities p_0 .. p_{L-1} */
  uint64_t seed;
  const int8_t *schedule; /* [schedule_steps][n_if] explicit delays */
  int32_t schedule_steps;
  int32_t at_order;       /* q, the number of past levels in Eq. (7); 0 = N_p + 1 */
  int32_t at_stencil;     /* buffer-element DoFs of Eq. (11) across delayed PE interfaces:
                             OR_AT_TEMPORAL: every mode from the q levels n-k .. n-k-q+1;
                             OR_AT_HYBRID: mode j from q_j = max(1, q - j) levels (the
                             spatio-temporal stencil of Sec. 3.3, see or_at_buffer) */
} or_config;

typedef struct or_solver or_solver;

/* Solver life cycle. w0 is [E][V][M]. max_steps bounds the stored history. */
int or_create(const or_config *cfg, const double *w0, int32_t max_steps, or_solver **out);
int or_step(or_solver *s, int32_t n_steps);
int or_get_state(const or_solver *s, double *w);
int64_t or_get_step(const or_solver *s);
int or_get_flags(const or_solver *s, int8_t *flags); /* troubled flags of the last limited stage */
int64_t or_total_flags(const or_solver *s);            /* troubled cells summed over all stages */
const char *or_error(const or_solver *s);
void or_destroy(or_solver *s);
int32_t or_n_interfaces(const or_solver *s);

/* Building blocks, exposed so tests can pin them one by one. */
double or_legendre(int j, double x);
double or_legendre_deriv(int j, int s, double x);   /* s-th derivative */
void or_gauss_legendre(int n, double *x, double *w);
int or_at_coeffs(int q, int k, double *c);          /* Eq. (8) solved exactly */
/* Buffer-element DoFs of Eq. (11) at level n from the modal data of the levels n-k, n-k-1, ...
   (levels[l] = [V][M] of level n-k-l, l < q): the temporal stencil (every mode from all q levels)
   or the hybrid one (mode j from the first max(1, q - j) levels with the weights of that order). */
int or_at_buffer(int q, int k, int V, int M, int hybrid, const double *levels, double *out);
uint64_t or_splitmix64(uint64_t x);
double or_saa_uniform(uint64_t seed, int64_t n, int32_t i, int32_t n_if);
int or_raw_delay(const or_config *cfg, int32_t n_if, int64_t n, int32_t i);
int or_eff_delay(const or_config *cfg, int32_t n_if, int64_t n, int32_t i);

int or_conv_flux(const or_config *cfg, const double *w, double *f);        /* f^c of Eq. (2) */
int or_source(const or_config *cfg, const double *w, double *s);           /* s of Eq. (2) */
int or_num_flux(const or_config *cfg, const double *wm, const double *wp, double *f);
int or_wave_speed(const or_config *cfg, const double *w, double *u, double *a);
int or_temperature(const or_config *cfg, const double *w, double *T, int *iters);
int or_pressure(const or_config *cfg, const double *w, double *p);
void or_species_thermo(const or_config *cfg, int i, double T, double *cp_R, double *h_RT, double *s_R);
int or_reaction_rates(const or_config *cfg, const double *w, double *kf, double *kr, double *qr);
int or_diff_flux(const or_config *cfg, const double *w, const double *dwdx, double *fd);
int or_char_matrices(const or_config *cfg, const double *wbar, double *Lm, double *Rm);
int or_weno_cell(const or_config *cfg, const double *wl, const double *wc, const double *wr, double *out);
void or_beta_matrix(int np, double *B);
void or_translation(int np, int side, double *T);
int or_rhs_sync(const or_config *cfg, const double *w, double *rhs);
int or_gradient_sync(const or_config *cfg, const double *w, double *q);
/* Troubled-cell flag (0/1) of the cell we between nbL and nbR ([V][M] each). */
int or_indicator(const or_config *cfg, const double *nbL, const double *we, const double *nbR, int ghostL,
                 int ghostR);

#endif
