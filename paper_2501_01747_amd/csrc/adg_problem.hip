// Placement of one ADG problem in device memory and the construction of its
// kernel arguments (shared by the single-problem solver and the batch).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "adg_problem.hpp"

namespace adg {

// ------------------------------------------------------------- host tables

// Legendre P_j(x) and P_j'(x) by the three-term recurrence and the derivative
// identity P'_{j+1} = P'_{j-1} + (2j+1) P_j.
void legendre_all(int n, double x, double *P, double *dP) {
  P[0] = 1.0;
  dP[0] = 0.0;
  if (n > 1) { P[1] = x; dP[1] = 1.0; }
  for (int j = 1; j + 1 < n; ++j) {
    P[j + 1] = ((2 * j + 1) * x * P[j] - j * P[j - 1]) / (j + 1);
    dP[j + 1] = dP[j - 1] + (2 * j + 1) * P[j];
  }
}

// Gauss-Legendre nodes (ascending) and weights, Newton iteration on P_n.
void gauss(int n, double *x, double *w) {
  double P[16], dP[16];
  for (int i = 0; i < n; ++i) {
    double z = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 60; ++it) {
      legendre_all(n + 1, z, P, dP);
      double dz = P[n] / dP[n];
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    legendre_all(n + 1, z, P, dP);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dP[n] * dP[n]);
  }
}

// Derivative of a Legendre series: if g = sum c_k P_k then g' = sum d_k P_k with
// d_k = (2k+1) sum_{m > k, m - k odd} c_m.
void legendre_series_derivative(int n, const double *c, double *d) {
  for (int k = 0; k < n; ++k) {
    double s = 0.0;
    for (int m = k + 1; m < n; m += 2) s += c[m];
    d[k] = (2 * k + 1) * s;
  }
}

void build_tables(int M, Tables &tb) {
  std::memset(&tb, 0, sizeof tb);
  double x[kMaxQ], w[kMaxQ], P[16], dP[16];
  gauss(M, x, w);
  for (int q = 0; q < M; ++q) {
    legendre_all(M, x[q], P, dP);
    for (int j = 0; j < M; ++j) {
      tb.B[q][j] = P[j];
      tb.WG[q][j] = w[q] * dP[j];
      tb.WB[q][j] = w[q] * P[j];
    }
  }
  for (int j = 0; j < M; ++j)
    for (int k = 0; k < M; ++k) {
      double s = 0.0;
      for (int q = 0; q < M; ++q) {
        legendre_all(M, x[q], P, dP);
        s += w[q] * dP[j] * P[k];
      }
      tb.Dm[j][k] = s;
    }
  for (int r = 0; r < M + 2; ++r) {
    double Pr[kMaxM];
    for (int j = 0; j < M; ++j)
      Pr[j] = r < M ? tb.B[r][j] : r == M ? 1.0 : (j & 1 ? -1.0 : 1.0);   // P_j(+1) = 1, P_j(-1) = (-1)^j
    double ga = 0.0, gb = 0.0;
    for (int j = 0; j < M; ++j) {
      ga += (2 * j + 1) * Pr[j];
      gb += (j & 1 ? -1.0 : 1.0) * (2 * j + 1) * Pr[j];
    }
    tb.GA[r] = ga;
    tb.GB[r] = gb;
    for (int k = 0; k < M; ++k) {
      double g = 0.0;
      for (int j = 0; j < M; ++j) g += (2 * j + 1) * Pr[j] * tb.Dm[j][k];
      tb.GD[r][k] = g;
    }
  }
}

// Smoothness quadratic form sum_s 2^(2s-1) int P_a^(s) P_b^(s) (Legendre
// coefficient space, where int P_k P_l = 2/(2k+1) delta_kl) and the
// re-expansion matrices of the left/right neighbour polynomials.
void build_limiter_tables(int M, LimiterArgs &la) {
  std::memset(la.Bm, 0, sizeof la.Bm);
  for (int a = 0; a < M; ++a)
    for (int b = 0; b < M; ++b) {
      double ca[kMaxM] = {0}, cb[kMaxM] = {0}, da[kMaxM], db[kMaxM];
      ca[a] = 1.0;
      cb[b] = 1.0;
      double sum = 0.0;
      for (int s = 1; s < M; ++s) {
        legendre_series_derivative(M, ca, da);
        legendre_series_derivative(M, cb, db);
        std::memcpy(ca, da, sizeof ca);
        std::memcpy(cb, db, sizeof cb);
        double ip = 0.0;
        for (int k = 0; k < M; ++k) ip += ca[k] * cb[k] * 2.0 / (2 * k + 1);
        sum += std::ldexp(1.0, 2 * s - 1) * ip;
      }
      la.Bm[a][b] = sum;
    }
  double x[kMaxQ + 1], w[kMaxQ + 1], P[16], dP[16], Ps[16], dPs[16];
  gauss(M + 1, x, w);
  for (int side = -1; side <= 1; side += 2) {
    double(*T)[kMaxM] = side < 0 ? la.Tl : la.Tr;
    for (int k = 0; k < kMaxM; ++k)
      for (int j = 0; j < kMaxM; ++j) T[k][j] = 0.0;
    for (int k = 0; k < M; ++k)
      for (int j = 0; j < M; ++j) {
        double s = 0.0;
        for (int q = 0; q < M + 1; ++q) {
          legendre_all(M, x[q], P, dP);
          legendre_all(M, x[q] - 2.0 * side, Ps, dPs);
          s += w[q] * Ps[j] * P[k];
        }
        T[k][j] = s * (2 * k + 1) / 2.0;
      }
  }
}

bool make_layout(const adg_physics *ph, const adg_discretization *d, const adg_async *as, Layout &L,
                 std::string *why, bool batched) {
  auto bad = [&](const char *m) { if (why) *why = m; return false; };
  if (!ph || !d || !as) return bad("null argument");
  if (d->order_p < 1 || d->order_p > 4) return bad("order_p must be 1..4");
  if (d->n_quad != 0 && d->n_quad != d->order_p + 1) return bad("n_quad must be 0 or order_p + 1");
  if (d->n_elem < 1) return bad("n_elem must be >= 1");
  if (!(d->dt > 0.0)) return bad("dt must be > 0");
  if (!(d->x_right > d->x_left)) return bad("x_right must exceed x_left");
  if (as->n_pe < 1 || as->n_pe > d->n_elem) return bad("n_pe must be in 1..n_elem");
  if (as->mode < 0 || as->mode > 3) return bad("unknown delay mode");
  if (as->mode != ADG_SYNC && (as->L < 1 || as->L > kMaxL)) return bad("L must be in 1..8");
  if (as->at_order < 0 || as->at_order > kMaxAT) return bad("at_order must be 0..6");
  if (ph->model == ADG_ONESTEP) {
    if (ph->n_species != 2) return bad("the one-step model has 2 species");
  } else if (ph->model == ADG_DETAILED) {
    if (!ph->mech) return bad("detailed model needs a mechanism");
    if (ph->n_species != ph->mech->n_species) return bad("n_species differs from the mechanism");
    if (ph->n_species < 1 || ph->n_species > kNsWideSpecies) return bad("the detailed model takes 1..16 species");
    if (d->limiter) return bad("the limiter supports the one-step model only");
    if (d->flux != ADG_RUSANOV) return bad("the detailed model uses the Rusanov flux");
  } else {
    return bad("unknown model");
  }
  if (d->rk != ADG_SSPRK3 && d->rk != ADG_RK2 && d->rk != ADG_LSERK4) return bad("unknown integrator");
  if (d->precision != ADG_FP64 && d->precision != ADG_MIXED_FP32 && d->precision != ADG_MIXED_BF16)
    return bad("unknown precision");
  if (d->limiter && d->indicator != ADG_KXRCF && d->indicator != ADG_MINMOD && d->indicator != ADG_ALL_CELLS)
    return bad("unknown indicator");
  if (as->at_stencil != ADG_AT_TEMPORAL && as->at_stencil != ADG_AT_HYBRID) return bad("unknown at_stencil");
  if (d->limiter && !(d->tvb_m >= 0.0)) return bad("tvb_m must be >= 0");
  if (as->mode == ADG_SAA) {
    if (!as->pmf) return bad("SAA needs pmf");
    double s = 0.0;
    for (int k = 0; k < as->L; ++k) {
      if (!(as->pmf[k] >= 0.0)) return bad("pmf entries must be >= 0");
      s += as->pmf[k];
    }
    if (std::fabs(s - 1.0) > 1e-12) return bad("pmf must sum to 1");
  }
  if (d->bc != ADG_PERIODIC && d->bc != ADG_TRANSMISSIVE) return bad("unknown boundary condition");
  if (d->flux != ADG_RUSANOV && d->flux != ADG_HLLC) return bad("unknown numerical flux");
  if (d->limiter) {
    if (!(d->weno_eps > 0.0)) return bad("weno_eps must be > 0");
    for (int k = 0; k < 3; ++k)
      if (!(d->weno_gamma[k] > 0.0)) return bad("weno_gamma entries must be > 0");
  }
  if (as->mode == ADG_SCHEDULE) {
    if (!as->schedule || as->schedule_steps < 1) return bad("schedule missing");
    // every delay must be one of the L admissible ones: the history ring holds L - 1 + q levels
    const long long nif = d->bc == ADG_PERIODIC ? as->n_pe : as->n_pe - 1;
    for (long long t = 0; t < (long long)as->schedule_steps * nif; ++t)
      if (as->schedule[t] < 0 || as->schedule[t] >= as->L) return bad("schedule delays must be in 0..L-1");
  }
  const bool periodic = d->bc == ADG_PERIODIC;
  L.E = d->n_elem;
  L.M = d->order_p + 1;
  L.V = 3 + ph->n_species;
  L.nif = periodic ? as->n_pe : as->n_pe - 1;
  L.nfaces = periodic ? L.E : L.E + 1;
  L.q = as->at_order > 0 ? as->at_order : d->order_p + 1;
  L.S = rk_stages(d->rk);
  const int kmax = as->mode == ADG_SYNC ? 0 : as->L - 1;
  L.D = kmax + L.q;
  const bool visc = ph->model == ADG_DETAILED && ph->viscous;
  L.off_F = 0;
  L.off_Wc = L.V;
  L.off_U = 2 * L.V;
  L.rec = 2 * L.V + (d->limiter ? 2 * L.V * L.M : 0);
  (void)visc;
  size_t nstate = state_doubles(L.E, L.V * L.M) * sizeof(double);
  size_t off = 0;
  // a 2N scheme with the limiter keeps two registers (each stage writes the one it
  // does not read)
  L.nbuf = (d->limiter && ph->model == ADG_ONESTEP && rk_stage(d->rk, 0).two_n) ? 4 : 3;
  L.state = off;  off += L.nbuf * align256(nstate);
  L.flags = off;  off += align256((size_t)L.E);
  L.face_if = off; off += align256(sizeof(int) * (L.E + 1));
  L.counters = off; off += 256;
  L.ring = off;   off += align256(sizeof(double) * (size_t)L.D * L.S * (L.nif > 0 ? L.nif : 1) * L.rec);
  L.sched = off;  off += as->mode == ADG_SCHEDULE ? align256((size_t)as->schedule_steps * (L.nif > 0 ? L.nif : 1)) : 0;
  L.mech = off;   off += ph->model == ADG_DETAILED ? align256(ns_mech_bytes(ph->n_species)) : 0;
  // the AT combinations carried from launch to launch (two buffers of (E + 1) faces x 2 Vg)
  L.carry_at = !batched && ph->model == ADG_DETAILED && L.nif > 0;
  L.at = off;     off += L.carry_at ? 2 * align256(sizeof(double) * (size_t)(L.E + 1) * (2 * (3 + ph->n_species) + 1)) : 0;
  L.total = off;
  return true;
}


adg_status check_precision(const adg_physics *ph, const adg_discretization *d, std::string *why) {
  if (d->precision == ADG_MIXED_BF16) {
    if (why) *why = "ADG_MIXED_BF16 is not supported: BF16 operators would exceed the error budget";
    return ADG_ERR_UNSUPPORTED;
  }
  if (d->precision == ADG_MIXED_FP32 && ph->model != ADG_DETAILED) {
    if (why) *why = "the one-step model runs in FP64 only";
    return ADG_ERR_UNSUPPORTED;
  }
  return ADG_OK;
}

adg_status setup_problem(const adg_physics *phys, const adg_discretization *disc, const adg_async *as, char *base,
                         const Layout &L, Problem &P) {
  if (phys->model == ADG_DETAILED && !ns_supported(phys->n_species, phys->mech->n_reactions))
    return ADG_ERR_UNSUPPORTED;
  std::vector<int32_t> off(as->n_pe + 1);
  for (int p = 0; p <= as->n_pe; ++p)
    off[p] = as->pe_offsets ? as->pe_offsets[p] : (int32_t)(((int64_t)p * L.E) / as->n_pe);
  if (off[0] != 0 || off[as->n_pe] != L.E) return ADG_ERR_ARG;
  for (int p = 0; p < as->n_pe; ++p)
    if (off[p + 1] <= off[p]) return ADG_ERR_ARG;
  P = Problem{};
  P.phys = *phys;
  P.disc = *disc;
  P.as = *as;
  P.lay = L;
  P.base = base;
  size_t nstate = state_doubles(L.E, L.V * L.M) * sizeof(double);
  for (int b = 0; b < L.nbuf; ++b) P.W[b] = (double *)(base + L.state + b * align256(nstate));
  P.flags = (int8_t *)(base + L.flags);
  P.face_if = (int *)(base + L.face_if);
  P.step = (long long *)(base + L.counters);
  P.err = (int *)(base + L.counters + 64);
  P.flag_count = (unsigned long long *)(base + L.counters + 128);
  P.ring = (double *)(base + L.ring);
  if (L.carry_at) {
    P.at = (double *)(base + L.at);
    P.at_stride = align256(sizeof(double) * (size_t)(L.E + 1) * (2 * (3 + phys->n_species) + 1)) / sizeof(double);
  }

  const bool periodic = disc->bc == ADG_PERIODIC;
  std::vector<int> fif(L.E + 1, -1);
  if (periodic) {
    for (int p = 0; p < as->n_pe; ++p) fif[off[p]] = p;
    fif[L.E] = fif[0];
  } else {
    for (int p = 1; p < as->n_pe; ++p) fif[off[p]] = p - 1;
  }
  if (hipMemcpy(P.face_if, fif.data(), sizeof(int) * (L.E + 1), hipMemcpyHostToDevice) != hipSuccess)
    return ADG_ERR_HIP;

  DelayParams dl{};
  dl.mode = as->mode;
  dl.L = as->L > 0 ? as->L : 1;
  dl.nif = L.nif;
  dl.q = L.q;
  dl.seed = as->seed;
  dl.hybrid = as->at_stencil == ADG_AT_HYBRID;
  if (as->mode == ADG_SAA) {
    double cum = 0.0;
    for (int k = 0; k < as->L; ++k) { cum += as->pmf[k]; dl.cum[k] = cum; }
  }
  if (as->mode == ADG_SCHEDULE) {
    dl.sched = (const int8_t *)(base + L.sched);
    dl.sched_steps = as->schedule_steps;
    if (hipMemcpy(base + L.sched, as->schedule, (size_t)as->schedule_steps * L.nif, hipMemcpyHostToDevice) != hipSuccess)
      return ADG_ERR_HIP;
  }
  RingParams rp{};
  rp.base = P.ring;
  rp.D = L.D;
  rp.stages = L.S;
  rp.rec = L.rec;
  rp.off_F = L.off_F;
  rp.off_Wc = L.off_Wc;
  rp.off_U = L.off_U;
  const double dx = (disc->x_right - disc->x_left) / L.E;
  Tables tb;
  build_tables(L.M, tb);

  if (phys->model == ADG_ONESTEP) {
    EulerArgs &a = P.ea;
    a.face_if = P.face_if;
    a.step = P.step;
    a.err = P.err;
    a.target = kNoTarget;
    a.E = L.E;
    a.periodic = periodic;
    a.store_U = disc->limiter && L.nif > 0;
    a.kbuf = P.W[2];
    a.kout = P.W[2];
    a.alt = disc->limiter && !rk_stage(disc->rk, 0).two_n;
    for (int b = 0; b < 3; ++b) a.W[b] = P.W[b];
    a.rk = rk_stage(disc->rk, 0);
    a.dt = disc->dt;
    a.two_over_dx = 2.0 / dx;
    a.ph = {phys->gamma, phys->q_heat, phys->e_act, phys->k_pre};
    a.dl = dl;
    a.ring = rp;
    a.tb = tb;
    if (disc->limiter) {
      LimiterArgs &l = P.la;
      l.flags = P.flags;
      l.flag_count = P.flag_count;
      l.kx_h = std::pow(dx, 0.5 * (disc->order_p + 1));
      l.indicator = disc->indicator;
      l.tvb_mh2 = disc->tvb_m * dx * dx;
      for (int k = 0; k < 3; ++k) l.gam[k] = disc->weno_gamma[k];
      l.eps = disc->weno_eps;
      build_limiter_tables(L.M, l);
    }
  } else {
    adg_status rc = ns_setup(P.na, phys, disc, L.E, L.M, periodic, dx, dl, rp, tb, P.face_if, P.step, P.err,
                             (void *)(base + L.mech));
    if (rc != ADG_OK) return rc;
    for (int b = 0; b < 3; ++b) P.na.W[b] = P.W[b];
    P.na.kbuf = P.W[2];
    P.na.rk = rk_stage(disc->rk, 0);
    P.na.target = kNoTarget;
    P.na.nst = L.S;
    P.na.at_in = nullptr;
    P.na.at_out = nullptr;
  }
  return ADG_OK;
}

hipError_t upload_state_host(const Problem &P, const double *w, hipStream_t st) {
  const Layout &L = P.lay;
  const int VM = L.V * L.M;
  std::vector<double> planes(state_doubles(L.E, VM), 0.0);
  for (int e = 0; e < L.E; ++e)
    for (int c = 0; c < VM; ++c) planes[sidx(e, c, VM)] = w[(size_t)e * VM + c];
  hipError_t e = hipMemcpyAsync(P.W[0], planes.data(), planes.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

hipError_t download_state_host(const Problem &P, const double *buf, double *w, hipStream_t st) {
  const Layout &L = P.lay;
  const int VM = L.V * L.M;
  std::vector<double> planes(state_doubles(L.E, VM));
  hipError_t e = hipMemcpyAsync(planes.data(), buf, planes.size() * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  for (int el = 0; el < L.E; ++el)
    for (int c = 0; c < VM; ++c) w[(size_t)el * VM + c] = planes[sidx(el, c, VM)];
  return hipSuccess;
}

// Zero fill by a kernel (not hipMemsetAsync): a caller may capture the reset of a problem into
// a HIP graph, and fill kernels replay like any other node.  Eight-byte words where the region
// is 8-byte aligned and long, single bytes otherwise (per-slot counters of a batch are 4-byte
// aligned).
__global__ void zero_words_kernel(unsigned long long *__restrict__ p, size_t nwords, unsigned char *__restrict__ tail,
                                  int ntail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride) p[i] = 0ull;
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

__global__ void zero_bytes_kernel(unsigned char *__restrict__ p, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  const int threads = 256;
  if (((uintptr_t)p & 7) || bytes < 64) {
    size_t blocks = (bytes + threads - 1) / threads;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(zero_bytes_kernel, dim3((unsigned)blocks), dim3(threads), 0, st, (unsigned char *)p, bytes);
    return hipGetLastError();
  }
  const size_t nwords = bytes / 8;
  size_t blocks = (nwords + threads - 1) / threads;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)blocks), dim3(threads), 0, st, (unsigned long long *)p, nwords,
                     (unsigned char *)p + nwords * 8, (int)(bytes % 8));
  return hipGetLastError();
}

hipError_t reset_problem(const Problem &P, hipStream_t st) {
  const Layout &L = P.lay;
  hipError_t e = launch_zero(P.base + L.counters, 256, st);
  if (e == hipSuccess)
    e = launch_zero(P.ring, sizeof(double) * (size_t)L.D * L.S * (L.nif > 0 ? L.nif : 1) * L.rec, st);
  if (e == hipSuccess) e = launch_zero(P.flags, (size_t)L.E, st);
  return e;
}

}  // namespace adg
