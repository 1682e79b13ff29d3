// Device helpers of the ADG library: delay draw, AT weights, one-step
// reactive-Euler physics and the numerical fluxes.
#pragma once

#include "adg_internal.hpp"

namespace adg {

// SplitMix64 output function (Steele, Lea & Flood 2014).
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  unsigned long long z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Cross-lane moves by the data-parallel-primitive (DPP) modifier, without the LDS
// crossbar.  dpp_move<CTRL>(x) returns the x of the lane that CTRL selects (a lane
// with no source keeps its own x): quad permutations, row mirrors and the
// wavefront shifts.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const unsigned long long v = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)v, (int)(unsigned)v, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(v >> 32), (int)(unsigned)(v >> 32), CTRL, 0xF, 0xF,
                                             false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL>
__device__ __forceinline__ int dpp_move(int x) {
  return __builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false);
}
constexpr int kDppFromNext = 0x130;   // lane l takes lane l+1's value (wavefront shift)
constexpr int kDppFromPrev = 0x138;   // lane l takes lane l-1's value
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane l takes lane 7-l of its group of 8
constexpr int kDppMirror = 0x140;     // lane l takes lane 15-l of its group of 16

// n mod d for a step count n >= 0 and 0 < d: in 32-bit arithmetic while n fits
// (a 64-bit remainder by a run-time divisor is a long instruction sequence).
__device__ __forceinline__ int step_mod(long long n, int d) {
  return n >= 0 && n <= 0x7fffffffll ? (int)((unsigned)n % (unsigned)d) : (int)(n % d);
}

// Delay at PE interface i for time step n (Sec. 4), clamped so that all q
// levels n-k .. n-k-q+1 exist.  BRANCH_FREE: the SAA bin is counted over all
// kMaxL - 1 bin edges with the loads of every edge issued together (the
// detailed-chemistry load phase, where the draw sits between the loads and the
// barrier); otherwise the bins are searched in order (the one-step kernels,
// where most draws end at the first edges).  Both give the same bin: the first
// j with u < cum[j] (cum is non-decreasing), at most L - 1.
template <bool BRANCH_FREE = false>
__device__ __forceinline__ int eff_delay(const DelayParams &d, long long n, int i) {
  int k = 0;
  if (d.mode == 1) {
    k = step_mod(n, d.L);
  } else if (d.mode == 2) {
    unsigned long long ctr = (unsigned long long)n * (unsigned long long)d.nif + (unsigned long long)i;
    unsigned long long z = splitmix64(d.seed ^ (ctr * 0x9E3779B97F4A7C15ull));
    double u = (double)(z >> 11) * 0x1.0p-53;
    if constexpr (BRANCH_FREE) {
#pragma unroll
      for (int j = 0; j < kMaxL - 1; ++j) k += (j < d.L - 1 && u >= d.cum[j]) ? 1 : 0;
    } else {
      k = d.L - 1;
      for (int j = 0; j < d.L; ++j)
        if (u < d.cum[j]) { k = j; break; }
    }
  } else if (d.mode == 3) {
    k = d.sched[(long long)step_mod(n, d.sched_steps) * d.nif + i];
  }
  if (k <= 0) return 0;
  long long lim = n - d.q + 1;
  if (lim < 0) lim = 0;
  return k > lim ? (int)lim : k;
}

// Weight of level n-k-j in the AT combination of Eq. (7): the Lagrange
// extrapolation weight prod_{m != j} (k+m)/(m-j), which is the solution of
// Eq. (8).  Exact: integer numerator and denominator, one rounding.
__device__ __forceinline__ double at_weight(int q, int k, int j) {
  long long num = 1, den = 1;
  for (int m = 0; m < q; ++m) {
    if (m == j) continue;
    num *= (long long)(k + m);
    den *= (long long)(m - j);
  }
  return (double)num / (double)den;
}

// Weight of level n-k-l for Legendre mode j of a buffer element (Eq. (11)): the temporal
// stencil uses all q levels for every mode; the hybrid spatio-temporal one extrapolates mode j,
// which carries the factor dx^j, from q_j = max(1, q - j) levels with the weights of that order
// (0 for the levels it does not use).
__device__ __forceinline__ double buffer_weight(const DelayParams &d, int k, int j, int l) {
  const int qj = d.hybrid ? max(1, d.q - j) : d.q;
  return l < qj ? at_weight(qj, k, l) : 0.0;
}
__device__ __forceinline__ int buffer_levels(const DelayParams &d, int j) { return d.hybrid ? max(1, d.q - j) : d.q; }

// End of time step n in the step's last launch (parity par): the next step's
// count goes to the other parity's counter.  Every launch of step n reads
// step[par] only, so one workgroup's plain store needs no atomic, no barrier and
// no wait; the next step's launches read it after this launch has ended.
__device__ __forceinline__ void advance_step(long long *step, int par, long long n, bool first_workgroup) {
  if (first_workgroup && threadIdx.x == 0) step[par ^ 1] = n + 1;
}

// ---------------------------------------------------------------- one-step model
struct Prim1 {
  double rho, u, p, T, a;
};

// rho E = rho u^2/2 + p/(gamma-1) + q rho Y_R;  T = p/rho (R = 1).
__device__ __forceinline__ bool prim1(const OneStep &ph, const double *w, Prim1 &pr) {
  pr.rho = w[0];
  const double rinv = 1.0 / pr.rho;
  pr.u = w[1] * rinv;
  pr.p = (ph.gamma - 1.0) * (w[2] - 0.5 * w[1] * pr.u - ph.q_heat * w[3]);
  pr.T = pr.p * rinv;
  pr.a = sqrt(ph.gamma * pr.T);
  return pr.rho > 0.0 && pr.p > 0.0 && isfinite(pr.p) && isfinite(pr.rho);
}

__device__ __forceinline__ void flux1(const double *w, const Prim1 &pr, double *f) {
  f[0] = w[1];
  f[1] = w[1] * pr.u + pr.p;
  f[2] = pr.u * (w[2] + pr.p);
  f[3] = w[3] * pr.u;
  f[4] = w[4] * pr.u;
}

// Local Lax-Friedrichs flux of Sec. 3.1.
__device__ __forceinline__ bool rusanov1(const OneStep &ph, const double *wm, const double *wp, double *f) {
  Prim1 pm, pp;
  bool ok = prim1(ph, wm, pm);
  ok = prim1(ph, wp, pp) && ok;
  double fm[5], fp[5];
  flux1(wm, pm, fm);
  flux1(wp, pp, fp);
  double lm = fabs(pm.u) + pm.a, lp = fabs(pp.u) + pp.a;
  double lam = lm > lp ? lm : lp;
#pragma unroll
  for (int v = 0; v < 5; ++v) f[v] = 0.5 * (fm[v] + fp[v] - lam * (wp[v] - wm[v]));
  return ok;
}

// HLLC (Toro, Spruce & Speares 1994) with Davis wave-speed bounds.
__device__ __forceinline__ bool hllc1(const OneStep &ph, const double *wm, const double *wp, double *f) {
  Prim1 pm, pp;
  bool ok = prim1(ph, wm, pm);
  ok = prim1(ph, wp, pp) && ok;
  double SL = fmin(pm.u - pm.a, pp.u - pp.a);
  double SR = fmax(pm.u + pm.a, pp.u + pp.a);
  if (SL >= 0.0) { flux1(wm, pm, f); return ok; }
  if (SR <= 0.0) { flux1(wp, pp, f); return ok; }
  double num = pp.p - pm.p + pm.rho * pm.u * (SL - pm.u) - pp.rho * pp.u * (SR - pp.u);
  double den = pm.rho * (SL - pm.u) - pp.rho * (SR - pp.u);
  double Ss = num / den;
  const bool left = Ss >= 0.0;
  const double *wk = left ? wm : wp;
  const Prim1 &pk = left ? pm : pp;
  const double Sk = left ? SL : SR;
  double fk[5];
  flux1(wk, pk, fk);
  double fac = pk.rho * (Sk - pk.u) / (Sk - Ss);
  double ws[5];
  ws[0] = fac;
  ws[1] = fac * Ss;
  ws[2] = fac * (wk[2] / pk.rho + (Ss - pk.u) * (Ss + pk.p / (pk.rho * (Sk - pk.u))));
  ws[3] = fac * (wk[3] / pk.rho);
  ws[4] = fac * (wk[4] / pk.rho);
#pragma unroll
  for (int v = 0; v < 5; ++v) f[v] = fk[v] + Sk * (ws[v] - wk[v]);
  return ok;
}

template <int FLUX>
__device__ __forceinline__ bool numflux1(const OneStep &ph, const double *wm, const double *wp, double *f) {
  if constexpr (FLUX == 1) return hllc1(ph, wm, wp, f);
  else return rusanov1(ph, wm, wp, f);
}

}  // namespace adg
