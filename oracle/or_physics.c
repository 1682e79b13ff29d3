/*
 * ADG oracle — test infrastructure only.
 *
 * Point-wise physics of Sec. 2: conserved variables, convective flux, diffusive
 * flux and chemical source of Eq. (1)-(3), the energy relation
 * E = u^2/2 - P/rho + h, and the two numerical fluxes of Sec. 3.1
 * (local Lax-Friedrichs and HLLC).
 *
 * Two models:
 *   one-step   nondimensional reactive Euler, R = 1, calorically perfect,
 *              species (R, P), h_R - h_P = q_heat, rate K rho Y_R exp(-Ea/T).
 *   detailed   thermally perfect mixture with NASA 7-coefficient thermo,
 *              reversible mass-action kinetics (equilibrium constants from the
 *              Gibbs energies), power-law viscosity, Pr and Le = 1 transport.
 *
 * Pins (tests/test_oracle_solver.py, tests/test_oracle_limiter.py,
 * tests/test_oracle_chemistry.py, tests/test_oracle_transport.py):
 *   fluxes     f_hat(w, w) = f(w); HLLC keeps a stationary contact; L A R = Lambda
 *              with A from finite differences of the flux
 *   thermo     dh/dT = cp and ds/dT = cp/T (finite differences); T(e(T)) = T
 *   kinetics   mass and element conservation of the production rates; zero net
 *              rate at an equilibrium composition; van 't Hoff relation for K_c;
 *              Arrhenius parameters recovered from rates at several T
 *   transport  linear theory of small modes on a periodic domain: an isobaric
 *              temperature mode decays at chi k^2 (heat conduction); a sound wave
 *              at k^2/2 (4 nu/3 + (gamma-1) chi) (the 4/3 of the stress); a
 *              composition mode of two thermodynamically identical species at
 *              D k^2 (J_i = -rho D dY_i/dx); with different formation enthalpies
 *              the same mode stays isothermal (the enthalpy flux sum h_i J_i)
 */
#include <math.h>
#include <string.h>

#include "or_internal.h"

/* ------------------------------------------------------------------ thermo */

/* NASA 7-coefficient polynomials: cp/R, h/(R T), s/R of species i at T. */
void or_species_thermo(const or_config *cfg, int i, double T, double *cp_R, double *h_RT, double *s_R) {
  const double *a = cfg->nasa7 + 7 * i;
  double T2 = T * T, T3 = T2 * T, T4 = T3 * T;
  if (cp_R) *cp_R = a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4;
  if (h_RT) *h_RT = a[0] + a[1] * T / 2.0 + a[2] * T2 / 3.0 + a[3] * T3 / 4.0 + a[4] * T4 / 5.0 + a[5] / T;
  if (s_R) *s_R = a[0] * log(T) + a[1] * T + a[2] * T2 / 2.0 + a[3] * T3 / 3.0 + a[4] * T4 / 4.0 + a[6];
}

/* Mixture specific internal energy and cv at T (per unit mass). */
static void mixture_e_cv(const or_config *cfg, const double *Y, double T, double *e, double *cv) {
  double es = 0.0, cvs = 0.0;
  for (int i = 0; i < cfg->n_species; ++i) {
    double cp_R, h_RT;
    or_species_thermo(cfg, i, T, &cp_R, &h_RT, NULL);
    double Ri = cfg->Ru / cfg->W[i];
    es += Y[i] * Ri * T * (h_RT - 1.0);
    cvs += Y[i] * Ri * (cp_R - 1.0);
  }
  *e = es;
  *cv = cvs;
}

/* Temperature from the internal energy e* = E - u^2/2 by Newton's method on
   sum_i Y_i e_i(T) = e*, from the fixed start T_guess, until |dT| <= 1e-12 T. */
static int newton_T(const or_config *cfg, const double *Y, double e_star, double *T_out, int *iters) {
  double T = cfg->T_guess;
  for (int it = 1; it <= 50; ++it) {
    double e, cv;
    mixture_e_cv(cfg, Y, T, &e, &cv);
    double dT = (e - e_star) / cv;
    T -= dT;
    if (!(T > 0.0) || !isfinite(T)) return -1;
    if (fabs(dT) <= 1e-12 * T) {
      *T_out = T;
      if (iters) *iters = it;
      return 0;
    }
  }
  return -1;
}

/* Primitive variables at one point.  Returns -1 for a non-physical state
   (rho <= 0, p <= 0, non-finite, or no Newton convergence). */
int or_primitives(const or_config *cfg, const double *w, or_prim *pr) {
  int ns = cfg->n_species;
  double rho = w[0];
  if (!(rho > 0.0) || !isfinite(rho)) return -1;
  pr->rho = rho;
  pr->u = w[1] / rho;
  for (int i = 0; i < ns; ++i) pr->Y[i] = w[3 + i] / rho;
  if (cfg->model == OR_ONESTEP) {
    /* rho E = rho u^2/2 + p/(gamma-1) + q rho Y_R: E = u^2/2 - p/rho + h with
       h = cp T + q Y_R and p = rho T. */
    double p = (cfg->gamma - 1.0) * (w[2] - 0.5 * rho * pr->u * pr->u - cfg->q_heat * w[3]);
    if (!(p > 0.0) || !isfinite(p)) return -1;
    pr->p = p;
    pr->T = p / rho;
    pr->a = sqrt(cfg->gamma * p / rho);
    return 0;
  }
  double e_star = w[2] / rho - 0.5 * pr->u * pr->u;
  double T;
  if (newton_T(cfg, pr->Y, e_star, &T, NULL) != 0) return -1;
  pr->T = T;
  double cp = 0.0, cv = 0.0, sum_YW = 0.0;
  for (int i = 0; i < ns; ++i) {
    double cp_R, h_RT;
    or_species_thermo(cfg, i, T, &cp_R, &h_RT, NULL);
    double Ri = cfg->Ru / cfg->W[i];
    pr->h_sp[i] = Ri * T * h_RT;
    pr->e_sp[i] = Ri * T * (h_RT - 1.0);
    cp += pr->Y[i] * Ri * cp_R;
    cv += pr->Y[i] * Ri * (cp_R - 1.0);
    sum_YW += pr->Y[i] / cfg->W[i];
  }
  pr->cp = cp;
  pr->cv = cv;
  pr->p = rho * cfg->Ru * T * sum_YW;
  if (!(pr->p > 0.0) || !isfinite(pr->p)) return -1;
  pr->a = sqrt(cp / cv * pr->p / rho);   /* frozen sound speed */
  return 0;
}

int or_temperature(const or_config *cfg, const double *w, double *T, int *iters) {
  if (cfg->model == OR_ONESTEP) {
    or_prim pr;
    if (or_primitives(cfg, w, &pr)) return -1;
    *T = pr.T;
    if (iters) *iters = 0;
    return 0;
  }
  double rho = w[0], u = w[1] / rho, Y[OR_MAXNS];
  for (int i = 0; i < cfg->n_species; ++i) Y[i] = w[3 + i] / rho;
  return newton_T(cfg, Y, w[2] / rho - 0.5 * u * u, T, iters);
}

int or_pressure(const or_config *cfg, const double *w, double *p) {
  or_prim pr;
  if (or_primitives(cfg, w, &pr)) return -1;
  *p = pr.p;
  return 0;
}

int or_wave_speed(const or_config *cfg, const double *w, double *u, double *a) {
  or_prim pr;
  if (or_primitives(cfg, w, &pr)) return -1;
  *u = pr.u;
  *a = pr.a;
  return 0;
}

/* -------------------------------------------------------- convective flux */

/* f^c = (rho u, rho u^2 + P, u (rho E + P), rho u Y_i), Eq. (2). */
void or_flux_from_prim(const or_config *cfg, const double *w, const or_prim *pr, double *f) {
  double u = pr->u;
  f[0] = w[1];
  f[1] = w[1] * u + pr->p;
  f[2] = u * (w[2] + pr->p);
  for (int i = 0; i < cfg->n_species; ++i) f[3 + i] = w[3 + i] * u;
}

int or_conv_flux(const or_config *cfg, const double *w, double *f) {
  or_prim pr;
  if (or_primitives(cfg, w, &pr)) return -1;
  or_flux_from_prim(cfg, w, &pr, f);
  return 0;
}

/* ------------------------------------------------------------- source s */

/* Forward/reverse rate constants and net rate of progress of each reaction of
   the detailed mechanism at the state w (mol / (m^3 s)). */
static void rates_detailed(const or_config *cfg, const double *w, const or_prim *pr,
                           double *kf_out, double *kr_out, double *q_out) {
  int ns = cfg->n_species;
  double T = pr->T, conc[OR_MAXNS], g_RT[OR_MAXNS];
  for (int i = 0; i < ns; ++i) {
    double h_RT, s_R;
    or_species_thermo(cfg, i, T, NULL, &h_RT, &s_R);
    g_RT[i] = h_RT - s_R;
    conc[i] = w[3 + i] / cfg->W[i];
  }
  for (int r = 0; r < cfg->n_reactions; ++r) {
    const int32_t *nf = cfg->nu_f + r * ns, *nr = cfg->nu_r + r * ns;
    double kf = cfg->A[r] * pow(T, cfg->b[r]) * exp(-cfg->Ea[r] / (cfg->Ru * T));
    double dG = 0.0;
    int dnu = 0;
    for (int i = 0; i < ns; ++i) {
      dG += (nr[i] - nf[i]) * g_RT[i];
      dnu += nr[i] - nf[i];
    }
    /* K_c = K_p (p_ref / (Ru T))^{sum nu}, K_p = exp(-Delta G / (Ru T)). */
    double Kc = exp(-dG) * pow(cfg->p_ref / (cfg->Ru * T), (double)dnu);
    double kr = kf / Kc;
    double fwd = kf, rev = kr;
    for (int i = 0; i < ns; ++i) {
      for (int m = 0; m < nf[i]; ++m) fwd *= conc[i];
      for (int m = 0; m < nr[i]; ++m) rev *= conc[i];
    }
    if (kf_out) kf_out[r] = kf;
    if (kr_out) kr_out[r] = kr;
    if (q_out) q_out[r] = fwd - rev;
  }
}

int or_reaction_rates(const or_config *cfg, const double *w, double *kf, double *kr, double *qr) {
  or_prim pr;
  if (cfg->model != OR_DETAILED) return -1;
  if (or_primitives(cfg, w, &pr)) return -1;
  rates_detailed(cfg, w, &pr, kf, kr, qr);
  return 0;
}

/* s = (0, 0, 0, W_i omega_i), Eq. (2). */
int or_source_from_prim(const or_config *cfg, const double *w, const or_prim *pr, double *s) {
  int ns = cfg->n_species;
  s[0] = s[1] = s[2] = 0.0;
  if (cfg->model == OR_ONESTEP) {
    double rate = cfg->k_pre * w[3] * exp(-cfg->e_act / pr->T);
    s[3] = -rate;
    s[4] = rate;
    for (int i = 2; i < ns; ++i) s[3 + i] = 0.0;
    return 0;
  }
  double q[OR_MAXR];
  rates_detailed(cfg, w, pr, NULL, NULL, q);
  for (int i = 0; i < ns; ++i) {
    double wdot = 0.0;
    for (int r = 0; r < cfg->n_reactions; ++r)
      wdot += (cfg->nu_r[r * ns + i] - cfg->nu_f[r * ns + i]) * q[r];
    s[3 + i] = cfg->W[i] * wdot;
  }
  return 0;
}

int or_source(const or_config *cfg, const double *w, double *s) {
  or_prim pr;
  if (or_primitives(cfg, w, &pr)) return -1;
  return or_source_from_prim(cfg, w, &pr, s);
}

/* --------------------------------------------------------- diffusive flux */

/* f^d = (0, tau, tau u - q, -rho Y_i V_i) of Eq. (2)-(3), with dw/dx the LDG
   auxiliary variable q = dw/dx of Sec. 3.1.  Transport reading: Le = 1, so
   every species has rho D = k / cp, and with the usual correction velocity the
   diffusive mass flux reduces to J_i = -rho D dY_i/dx (sum J_i = 0). */
void or_diff_flux_from_prim(const or_config *cfg, const double *w, const or_prim *pr,
                            const double *dwdx, double *fd) {
  int ns = cfg->n_species;
  double rho = pr->rho, u = pr->u;
  double mu = cfg->mu_ref * pow(pr->T / cfg->T_ref, cfg->mu_exp);
  double kappa = mu * pr->cp / cfg->prandtl;
  double rhoD = kappa / pr->cp;
  double u_x = (dwdx[1] - u * dwdx[0]) / rho;
  double E = w[2] / rho;
  double E_x = (dwdx[2] - E * dwdx[0]) / rho;
  double e_x = E_x - u * u_x;
  double Y_x[OR_MAXNS], sum_eY = 0.0;
  for (int i = 0; i < ns; ++i) {
    Y_x[i] = (dwdx[3 + i] - pr->Y[i] * dwdx[0]) / rho;
    sum_eY += pr->e_sp[i] * Y_x[i];
  }
  double T_x = (e_x - sum_eY) / pr->cv;
  double tau = 4.0 / 3.0 * mu * u_x;
  double qh = -kappa * T_x;
  double J[OR_MAXNS];
  for (int i = 0; i < ns; ++i) {
    J[i] = -rhoD * Y_x[i];
    qh += pr->h_sp[i] * J[i];
  }
  fd[0] = 0.0;
  fd[1] = tau;
  fd[2] = tau * u - qh;
  for (int i = 0; i < ns; ++i) fd[3 + i] = -J[i];
}

int or_diff_flux(const or_config *cfg, const double *w, const double *dwdx, double *fd) {
  or_prim pr;
  if (cfg->model != OR_DETAILED) return -1;
  if (or_primitives(cfg, w, &pr)) return -1;
  or_diff_flux_from_prim(cfg, w, &pr, dwdx, fd);
  return 0;
}

/* ------------------------------------------------------- numerical fluxes */

/* Local Lax-Friedrichs flux f = (f- + f+ - lambda (w+ - w-)) / 2 with lambda the
   larger spectral radius |u| + a of the flux Jacobian at the two traces. */
static int rusanov(const or_config *cfg, const double *wm, const double *wp, double *f) {
  int V = 3 + cfg->n_species;
  or_prim pm, pp;
  if (or_primitives(cfg, wm, &pm) || or_primitives(cfg, wp, &pp)) return -1;
  double fm[OR_MAXV], fp[OR_MAXV];
  or_flux_from_prim(cfg, wm, &pm, fm);
  or_flux_from_prim(cfg, wp, &pp, fp);
  double lm = fabs(pm.u) + pm.a, lp = fabs(pp.u) + pp.a;
  double lam = lm > lp ? lm : lp;
  for (int v = 0; v < V; ++v) f[v] = 0.5 * (fm[v] + fp[v] - lam * (wp[v] - wm[v]));
  return 0;
}

/* HLLC (Toro, Spruce & Speares 1994) with the Davis wave-speed bounds
   S_L = min(u- - a-, u+ - a+), S_R = max(u- + a-, u+ + a+); the species are
   carried by the contact. */
static int hllc(const or_config *cfg, const double *wm, const double *wp, double *f) {
  int V = 3 + cfg->n_species;
  or_prim pm, pp;
  if (or_primitives(cfg, wm, &pm) || or_primitives(cfg, wp, &pp)) return -1;
  double SL = fmin(pm.u - pm.a, pp.u - pp.a);
  double SR = fmax(pm.u + pm.a, pp.u + pp.a);
  double fm[OR_MAXV], fp[OR_MAXV];
  if (SL >= 0.0) {
    or_flux_from_prim(cfg, wm, &pm, f);
    return 0;
  }
  if (SR <= 0.0) {
    or_flux_from_prim(cfg, wp, &pp, f);
    return 0;
  }
  double num = pp.p - pm.p + pm.rho * pm.u * (SL - pm.u) - pp.rho * pp.u * (SR - pp.u);
  double den = pm.rho * (SL - pm.u) - pp.rho * (SR - pp.u);
  double Ss = num / den;
  const double *wk;
  const or_prim *pk;
  double Sk, *fk;
  if (Ss >= 0.0) {
    wk = wm; pk = &pm; Sk = SL; fk = fm;
  } else {
    wk = wp; pk = &pp; Sk = SR; fk = fp;
  }
  or_flux_from_prim(cfg, wk, pk, fk);
  double fac = pk->rho * (Sk - pk->u) / (Sk - Ss);
  double ws[OR_MAXV];
  ws[0] = fac;
  ws[1] = fac * Ss;
  ws[2] = fac * (wk[2] / pk->rho + (Ss - pk->u) * (Ss + pk->p / (pk->rho * (Sk - pk->u))));
  for (int i = 0; i < cfg->n_species; ++i) ws[3 + i] = fac * pk->Y[i];
  for (int v = 0; v < V; ++v) f[v] = fk[v] + Sk * (ws[v] - wk[v]);
  return 0;
}

int or_num_flux(const or_config *cfg, const double *wm, const double *wp, double *f) {
  return cfg->flux == OR_HLLC ? hllc(cfg, wm, wp, f) : rusanov(cfg, wm, wp, f);
}
