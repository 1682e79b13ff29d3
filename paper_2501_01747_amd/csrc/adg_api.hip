// Host runtime of the ADG library: the C ABI of include/adg.h.
//
// The solver owns no device memory: the caller's workspace is carved into
// 256-byte aligned regions (state planes, limiter buffers, history ring, face
// map, counters).  Every launch goes to the caller's stream; adg_set_graph()
// switches adg_step to a captured HIP graph of several time steps.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "adg.h"
#include "adg_internal.hpp"
#include "adg_ns.hpp"

using namespace adg;

namespace {

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

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t state, wlim, flags, face_if, counters, ring, sched, mech, total;
  int nif, nfaces, D, rec, q, V, M, E;
  int off_F, off_Wc, off_U;
};

bool make_layout(const adg_physics *ph, const adg_discretization *d, const adg_async *as, Layout &L,
                 std::string *why) {
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
    if (d->limiter) return bad("the limiter supports the one-step model only");
    if (d->flux != ADG_RUSANOV) return bad("the detailed model uses the Rusanov flux");
  } else {
    return bad("unknown model");
  }
  if (as->mode == ADG_SAA) {
    if (!as->pmf) return bad("SAA needs pmf");
    double s = 0.0;
    for (int k = 0; k < as->L; ++k) {
      if (!(as->pmf[k] >= 0.0)) return bad("pmf entries must be >= 0");
      s += as->pmf[k];
    }
    if (std::fabs(s - 1.0) > 1e-12) return bad("pmf must sum to 1");
  }
  if (as->mode == ADG_SCHEDULE && (!as->schedule || as->schedule_steps < 1)) return bad("schedule missing");
  const bool periodic = d->bc == ADG_PERIODIC;
  L.E = d->n_elem;
  L.M = d->order_p + 1;
  L.V = 3 + ph->n_species;
  L.nif = periodic ? as->n_pe : as->n_pe - 1;
  L.nfaces = periodic ? L.E : L.E + 1;
  L.q = as->at_order > 0 ? as->at_order : d->order_p + 1;
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
  L.state = off;  off += 3 * align256(nstate);
  L.wlim = off;   off += d->limiter ? align256(nstate) : 0;
  L.flags = off;  off += align256((size_t)L.E);
  L.face_if = off; off += align256(sizeof(int) * (L.E + 1));
  L.counters = off; off += 256;
  L.ring = off;   off += align256(sizeof(double) * (size_t)L.D * 3 * (L.nif > 0 ? L.nif : 1) * L.rec);
  L.sched = off;  off += as->mode == ADG_SCHEDULE ? align256((size_t)as->schedule_steps * (L.nif > 0 ? L.nif : 1)) : 0;
  L.mech = off;   off += ph->model == ADG_DETAILED ? align256(sizeof(NsMech)) : 0;
  L.total = off;
  return true;
}

}  // namespace

struct adg_solver {
  adg_physics phys{};
  adg_discretization disc{};
  adg_async as{};
  Layout lay{};
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  double *W[3] = {nullptr, nullptr, nullptr};
  double *Wlim = nullptr;
  int8_t *flags = nullptr;
  int *face_if = nullptr;
  long long *step = nullptr;
  unsigned *done = nullptr;
  int *err = nullptr;
  unsigned long long *flag_count = nullptr;
  double *ring = nullptr;
  EulerArgs ea{};
  LimiterArgs la{};
  NsArgs na{};
  int graph_steps = 0;
  int graph_built_for = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;
  std::vector<hipEvent_t> prof_events;
  std::string msg;
};

namespace {

adg_status fail(adg_solver *s, adg_status code, const std::string &m) {
  if (s) s->msg = m;
  return code;
}

adg_status hip_fail(adg_solver *s, hipError_t e, const char *where) {
  return fail(s, ADG_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(s, expr)                          \
  do {                                            \
    hipError_t _e = (expr);                       \
    if (_e != hipSuccess) return hip_fail(s, _e, #expr); \
  } while (0)

// Launch the kernels of one time step.  `timer` (optional) records an event
// pair around each launch for adg_profile.
typedef void (*TimerFn)(adg_solver *, int cls, bool begin);

adg_status enqueue_step(adg_solver *s, hipStream_t st, TimerFn timer) {
  const int M = s->lay.M;
  const int in_buf[3] = {0, 1, 2}, out_buf[3] = {1, 2, 0};
  for (int stage = 0; stage < 3; ++stage) {
    if (s->phys.model == ADG_ONESTEP) {
      EulerArgs a = s->ea;
      a.w0 = s->W[0];
      a.ws = s->W[in_buf[stage]];
      a.wout = s->W[out_buf[stage]];
      a.stage = stage;
      a.advance = stage == 2 && !s->disc.limiter;
      if (timer) timer(s, 0, true);
      HIP_TRY(s, launch_euler_stage(M, s->disc.flux, a, st));
      if (timer) timer(s, 0, false);
      if (s->disc.limiter) {
        LimiterArgs l = s->la;
        l.w = s->W[out_buf[stage]];
        l.stage = stage;
        l.advance = 0;
        if (timer) timer(s, 1, true);
        HIP_TRY(s, launch_limiter(M, l, st));
        if (timer) timer(s, 1, false);
        l.advance = stage == 2;
        if (timer) timer(s, 2, true);
        HIP_TRY(s, launch_limiter_scatter(M, l, st));
        if (timer) timer(s, 2, false);
      }
    } else {
      NsArgs a = s->na;
      a.w0 = s->W[0];
      a.ws = s->W[in_buf[stage]];
      a.wout = s->W[out_buf[stage]];
      a.stage = stage;
      a.advance = stage == 2;
      if (timer) timer(s, 0, true);
      HIP_TRY(s, launch_ns_stage(M, a, st));
      if (timer) timer(s, 0, false);
    }
  }
  return ADG_OK;
}

void destroy_graph(adg_solver *s) {
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  s->gexec = nullptr;
  s->graph = nullptr;
  s->graph_built_for = 0;
}

adg_status build_graph(adg_solver *s) {
  destroy_graph(s);
  if (!s->cap_stream) HIP_TRY(s, hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  HIP_TRY(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
  adg_status rc = ADG_OK;
  for (int i = 0; i < s->graph_steps && rc == ADG_OK; ++i) rc = enqueue_step(s, s->cap_stream, nullptr);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
  if (rc != ADG_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
  if (e != hipSuccess) return hip_fail(s, e, "hipStreamEndCapture");
  s->graph = g;
  HIP_TRY(s, hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0));
  s->graph_built_for = s->graph_steps;
  return ADG_OK;
}

}  // namespace

extern "C" {

size_t adg_workspace_bytes(const adg_physics *phys, const adg_discretization *disc, const adg_async *as) {
  Layout L;
  if (!make_layout(phys, disc, as, L, nullptr)) return 0;
  return L.total;
}

adg_status adg_create(const adg_physics *phys, const adg_discretization *disc, const adg_async *as,
                      void *device_workspace, size_t workspace_bytes, void *hip_stream, adg_solver **out) {
  if (!out) return ADG_ERR_ARG;
  *out = nullptr;
  Layout L;
  std::string why;
  if (!make_layout(phys, disc, as, L, &why)) return ADG_ERR_ARG;
  if (!device_workspace || ((uintptr_t)device_workspace & 255)) return ADG_ERR_ARG;
  if (workspace_bytes < L.total) return ADG_ERR_NOMEM;
  if (phys->model == ADG_DETAILED && !ns_supported(phys->n_species, phys->mech->n_reactions))
    return ADG_ERR_UNSUPPORTED;
  std::vector<int32_t> off(as->n_pe + 1);
  for (int p = 0; p <= as->n_pe; ++p)
    off[p] = as->pe_offsets ? as->pe_offsets[p] : (int32_t)(((int64_t)p * L.E) / as->n_pe);
  if (off[0] != 0 || off[as->n_pe] != L.E) return ADG_ERR_ARG;
  for (int p = 0; p < as->n_pe; ++p)
    if (off[p + 1] <= off[p]) return ADG_ERR_ARG;

  adg_solver *s = new adg_solver();
  s->phys = *phys;
  s->disc = *disc;
  s->as = *as;
  s->lay = L;
  s->stream = (hipStream_t)hip_stream;
  s->ws = (char *)device_workspace;
  size_t nstate = state_doubles(L.E, L.V * L.M) * sizeof(double);
  for (int b = 0; b < 3; ++b) s->W[b] = (double *)(s->ws + L.state + b * align256(nstate));
  s->Wlim = disc->limiter ? (double *)(s->ws + L.wlim) : nullptr;
  s->flags = (int8_t *)(s->ws + L.flags);
  s->face_if = (int *)(s->ws + L.face_if);
  s->step = (long long *)(s->ws + L.counters);
  s->err = (int *)(s->ws + L.counters + 64);
  s->done = (unsigned *)(s->ws + L.counters + 192);
  s->flag_count = (unsigned long long *)(s->ws + L.counters + 128);
  s->ring = (double *)(s->ws + L.ring);

  const bool periodic = disc->bc == ADG_PERIODIC;
  std::vector<int> fif(L.E + 1, -1);
  if (periodic) {
    for (int p = 0; p < as->n_pe; ++p) fif[off[p]] = p;
    fif[L.E] = fif[0];
  } else {
    for (int p = 1; p < as->n_pe; ++p) fif[off[p]] = p - 1;
  }
  hipError_t e = hipMemcpy(s->face_if, fif.data(), sizeof(int) * (L.E + 1), hipMemcpyHostToDevice);
  if (e != hipSuccess) { delete s; return ADG_ERR_HIP; }

  DelayParams dl{};
  dl.mode = as->mode;
  dl.L = as->L > 0 ? as->L : 1;
  dl.nif = L.nif;
  dl.q = L.q;
  dl.seed = as->seed;
  if (as->mode == ADG_SAA) {
    double cum = 0.0;
    for (int k = 0; k < as->L; ++k) { cum += as->pmf[k]; dl.cum[k] = cum; }
  }
  if (as->mode == ADG_SCHEDULE) {
    dl.sched = (const int8_t *)(s->ws + L.sched);
    dl.sched_steps = as->schedule_steps;
    e = hipMemcpy(s->ws + L.sched, as->schedule, (size_t)as->schedule_steps * L.nif, hipMemcpyHostToDevice);
    if (e != hipSuccess) { delete s; return ADG_ERR_HIP; }
  }
  RingParams rp{};
  rp.base = s->ring;
  rp.D = L.D;
  rp.rec = L.rec;
  rp.off_F = L.off_F;
  rp.off_Wc = L.off_Wc;
  rp.off_U = L.off_U;
  const double dx = (disc->x_right - disc->x_left) / L.E;
  Tables tb;
  build_tables(L.M, tb);

  if (phys->model == ADG_ONESTEP) {
    EulerArgs &a = s->ea;
    a.face_if = s->face_if;
    a.step = s->step;
    a.done = s->done;
    a.err = s->err;
    a.E = L.E;
    a.periodic = periodic;
    a.store_U = disc->limiter && L.nif > 0;
    a.dt = disc->dt;
    a.two_over_dx = 2.0 / dx;
    a.ph = {phys->gamma, phys->q_heat, phys->e_act, phys->k_pre};
    a.dl = dl;
    a.ring = rp;
    a.tb = tb;
    if (disc->limiter) {
      LimiterArgs &l = s->la;
      l.wlim = s->Wlim;
      l.flags = s->flags;
      l.flag_count = s->flag_count;
      l.face_if = s->face_if;
      l.step = s->step;
      l.done = s->done;
      l.err = s->err;
      l.E = L.E;
      l.periodic = periodic;
      l.kx_h = std::pow(dx, 0.5 * (disc->order_p + 1));
      for (int k = 0; k < 3; ++k) l.gam[k] = disc->weno_gamma[k];
      l.eps = disc->weno_eps;
      l.ph = a.ph;
      l.dl = dl;
      l.ring = rp;
      l.tb = tb;
      build_limiter_tables(L.M, l);
    }
  } else {
    adg_status rc = ns_setup(s->na, phys, disc, L.E, L.M, periodic, dx, dl, rp, tb, s->face_if, s->step, s->done, s->err,
                             (NsMech *)(s->ws + L.mech));
    if (rc != ADG_OK) { delete s; return rc; }
  }
  *out = s;
  return ADG_OK;
}

adg_status adg_set_state(adg_solver *s, const double *w, int64_t count, int32_t where) {
  if (!s || !w) return ADG_ERR_ARG;
  const Layout &L = s->lay;
  const int VM = L.V * L.M;
  if (count != (int64_t)L.E * VM) return fail(s, ADG_ERR_ARG, "state size mismatch");
  if (where == ADG_HOST) {
    std::vector<double> planes(state_doubles(L.E, VM), 0.0);
    for (int e = 0; e < L.E; ++e)
      for (int c = 0; c < VM; ++c) planes[sidx(e, c, VM)] = w[(size_t)e * VM + c];
    HIP_TRY(s, hipMemcpyAsync(s->W[0], planes.data(), planes.size() * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
  } else if (where == ADG_DEVICE) {
    HIP_TRY(s, launch_to_planes(w, s->W[0], L.E, VM, s->stream));
  } else {
    return fail(s, ADG_ERR_ARG, "where must be ADG_HOST or ADG_DEVICE");
  }
  HIP_TRY(s, hipMemsetAsync(s->ws + L.counters, 0, 256, s->stream));
  HIP_TRY(s, hipMemsetAsync(s->ring, 0, sizeof(double) * (size_t)L.D * 3 * (L.nif > 0 ? L.nif : 1) * L.rec, s->stream));
  HIP_TRY(s, hipMemsetAsync(s->flags, 0, (size_t)L.E, s->stream));
  if (where == ADG_HOST) HIP_TRY(s, hipStreamSynchronize(s->stream));
  return ADG_OK;
}

adg_status adg_step(adg_solver *s, int32_t n_steps) {
  if (!s || n_steps < 0) return ADG_ERR_ARG;
  if (s->graph_steps > 0) {
    if (s->graph_built_for != s->graph_steps) {
      adg_status rc = build_graph(s);
      if (rc != ADG_OK) return rc;
    }
    int full = n_steps / s->graph_steps, rest = n_steps % s->graph_steps;
    for (int i = 0; i < full; ++i) HIP_TRY(s, hipGraphLaunch(s->gexec, s->stream));
    for (int i = 0; i < rest; ++i) {
      adg_status rc = enqueue_step(s, s->stream, nullptr);
      if (rc != ADG_OK) return rc;
    }
    return ADG_OK;
  }
  for (int i = 0; i < n_steps; ++i) {
    adg_status rc = enqueue_step(s, s->stream, nullptr);
    if (rc != ADG_OK) return rc;
  }
  return ADG_OK;
}

adg_status adg_sync(adg_solver *s) {
  if (!s) return ADG_ERR_ARG;
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  int err = 0;
  HIP_TRY(s, hipMemcpy(&err, s->err, sizeof(int), hipMemcpyDeviceToHost));
  if (err) return fail(s, ADG_ERR_STATE, "non-physical state (rho <= 0, p <= 0, non-finite or no T convergence)");
  return ADG_OK;
}

adg_status adg_get_state(adg_solver *s, double *w, int64_t count, int32_t where) {
  if (!s || !w) return ADG_ERR_ARG;
  const Layout &L = s->lay;
  const int VM = L.V * L.M;
  if (count != (int64_t)L.E * VM) return fail(s, ADG_ERR_ARG, "state size mismatch");
  if (where == ADG_HOST) {
    std::vector<double> planes(state_doubles(L.E, VM));
    HIP_TRY(s, hipMemcpyAsync(planes.data(), s->W[0], planes.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    for (int e = 0; e < L.E; ++e)
      for (int c = 0; c < VM; ++c) w[(size_t)e * VM + c] = planes[sidx(e, c, VM)];
  } else if (where == ADG_DEVICE) {
    HIP_TRY(s, launch_from_planes(s->W[0], w, L.E, VM, s->stream));
  } else {
    return fail(s, ADG_ERR_ARG, "where must be ADG_HOST or ADG_DEVICE");
  }
  return adg_sync(s);
}

adg_status adg_get_flags(adg_solver *s, int8_t *flags, int64_t *total) {
  if (!s) return ADG_ERR_ARG;
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  if (flags) HIP_TRY(s, hipMemcpy(flags, s->flags, (size_t)s->lay.E, hipMemcpyDeviceToHost));
  if (total) {
    unsigned long long c = 0;
    HIP_TRY(s, hipMemcpy(&c, s->flag_count, sizeof c, hipMemcpyDeviceToHost));
    *total = (int64_t)c;
  }
  return ADG_OK;
}

int64_t adg_step_count(adg_solver *s) {
  if (!s) return -1;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return -1;
  long long n = 0;
  if (hipMemcpy(&n, s->step, sizeof n, hipMemcpyDeviceToHost) != hipSuccess) return -1;
  return n;
}

int32_t adg_n_interfaces(const adg_solver *s) { return s ? s->lay.nif : -1; }

static void prof_timer(adg_solver *s, int cls, bool begin) {
  (void)cls;
  (void)begin;
  hipEvent_t ev;
  if (hipEventCreate(&ev) != hipSuccess) return;
  (void)hipEventRecord(ev, s->stream);
  s->prof_events.push_back(ev);
}

adg_status adg_profile(adg_solver *s, int32_t n_steps, double *ms_out, int64_t *launches_out, int32_t n_classes) {
  if (!s || n_steps < 1 || !ms_out || !launches_out || n_classes < 1) return ADG_ERR_ARG;
  s->prof_events.clear();
  for (int i = 0; i < n_steps; ++i) {
    adg_status rc = enqueue_step(s, s->stream, prof_timer);
    if (rc != ADG_OK) return rc;
  }
  // the launch classes of one step, in order
  std::vector<int> order;
  for (int stage = 0; stage < 3; ++stage) {
    order.push_back(0);
    if (s->phys.model == ADG_ONESTEP && s->disc.limiter) { order.push_back(1); order.push_back(2); }
  }
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  std::vector<double> sum(n_classes, 0.0);
  std::vector<int64_t> cnt(n_classes, 0);
  size_t per_step = order.size();
  for (int i = 0; i < n_steps; ++i)
    for (size_t k = 0; k < per_step; ++k) {
      size_t idx = ((size_t)i * per_step + k) * 2;
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, s->prof_events[idx], s->prof_events[idx + 1]);
      int c = order[k];
      if (c < n_classes) { sum[c] += ms; cnt[c] += 1; }
    }
  for (hipEvent_t ev : s->prof_events) (void)hipEventDestroy(ev);
  s->prof_events.clear();
  for (int c = 0; c < n_classes; ++c) {
    ms_out[c] = cnt[c] ? sum[c] / cnt[c] : 0.0;
    launches_out[c] = cnt[c];
  }
  return adg_sync(s);
}

adg_status adg_set_graph(adg_solver *s, int32_t steps_per_graph) {
  if (!s || steps_per_graph < 0) return ADG_ERR_ARG;
  s->graph_steps = steps_per_graph;
  if (steps_per_graph == 0) destroy_graph(s);
  return ADG_OK;
}

void adg_destroy(adg_solver *s) {
  if (!s) return;
  destroy_graph(s);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s;
}

const char *adg_last_error(const adg_solver *s) { return s ? s->msg.c_str() : "null solver"; }

}  // extern "C"
