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
#include <algorithm>
#include <string>
#include <vector>

#include "adg.h"
#include "adg_internal.hpp"
#include "adg_ns.hpp"
#include "adg_problem.hpp"

using namespace adg;

struct adg_solver {
  Problem P;
  hipStream_t stream = nullptr;
  int cur = 0;            // state buffer at the start of the next step (2N schemes alternate 0 and 1)
  int graph_cur = 0;      // state buffer the captured graph starts from
  int graph_cur_after = 0;
  int par = 0;            // step counter parity of the next step (P.step[par] holds its count)
  int graph_par = 0;      // parity the captured graph starts from
  int graph_par_after = 0;
  int ns_cfg = 0;   // work decomposition of the detailed-chemistry stage kernel
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
  const int M = s->P.lay.M, S = s->P.lay.S;
  const int rk = s->P.disc.rk;
  const int in_buf[3] = {0, 1, 2}, out_buf[3] = {1, 2, 0};
  for (int stage = 0; stage < S; ++stage) {
    const RkStage r = rk_stage(rk, stage);
    // Shu-Osher SSP-RK3: w^n in buffer 0, stages in 1 and 2, the last stage back into 0;
    // with the limiter no stage may write a buffer it reads, so w^n alternates between
    // buffers 0 and 1 (s->cur), stage 1 goes to the other one, stage 2 to buffer 2 and
    // stage 3 to the other one again.  2N schemes: the state alternates between buffers
    // 0 and 1 (s->cur holds it at the start of the step), the register is buffer 2
    // (with the limiter, buffers 2 and 3 alternate the same way).
    const bool alt = !r.two_n && s->P.disc.limiter && s->P.phys.model == ADG_ONESTEP;
    const int lim_in[3] = {s->cur, 1 - s->cur, 2}, lim_out[3] = {1 - s->cur, 2, 1 - s->cur};
    const int bi = r.two_n ? (s->cur + stage) % 2 : alt ? lim_in[stage] : in_buf[stage];
    const int bo = r.two_n ? (s->cur + stage + 1) % 2 : alt ? lim_out[stage] : out_buf[stage];
    const bool last = stage == S - 1;
    if (s->P.phys.model == ADG_ONESTEP) {
      const bool lim = s->P.disc.limiter != 0;
      EulerArgs a = s->P.ea;
      a.alt = 0;   // buffers chosen here (the batched kernels choose them by step parity)
      a.w0 = s->P.W[alt ? s->cur : 0];
      a.ws = s->P.W[bi];
      a.wout = s->P.W[bo];
      if (lim && r.two_n) {
        // the two registers alternate like the state: read W[2 + bi], write W[2 + bo]
        a.kbuf = s->P.W[2 + bi];
        a.kout = s->P.W[2 + bo];
      }
      a.stage = stage;
      a.rk = r;
      a.advance = last;
      a.par = s->par;
      if (timer) timer(s, 0, true);
      HIP_TRY(s, launch_euler_stage(M, s->P.disc.flux, a, lim ? &s->P.la : nullptr, st));
      if (timer) timer(s, 0, false);
    } else {
      NsArgs a = s->P.na;
      a.w0 = s->P.W[0];
      a.ws = s->P.W[bi];
      a.wout = s->P.W[bo];
      a.stage = stage;
      a.rk = r;
      a.advance = last;
      a.par = s->par;
      if (timer) timer(s, 0, true);
      HIP_TRY(s, launch_ns_stage(M, s->ns_cfg, a, st));
      if (timer) timer(s, 0, false);
    }
  }
  if (rk_stage(rk, 0).two_n) s->cur = (s->cur + S) % 2;
  else if (s->P.disc.limiter && s->P.phys.model == ADG_ONESTEP) s->cur = 1 - s->cur;
  s->par ^= 1;   // the step's last launch wrote the next count into the other counter
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
  const int cur0 = s->cur, par0 = s->par;
  for (int i = 0; i < s->graph_steps && rc == ADG_OK; ++i) rc = enqueue_step(s, s->cap_stream, nullptr);
  s->graph_cur = cur0;
  s->graph_cur_after = s->cur;
  s->graph_par = par0;
  s->graph_par_after = s->par;
  s->cur = cur0;   // nothing ran: capture only records
  s->par = par0;
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
  adg_solver *s = new adg_solver();
  adg_status rc = setup_problem(phys, disc, as, (char *)device_workspace, L, s->P);
  if (rc != ADG_OK) { delete s; return rc; }
  s->stream = (hipStream_t)hip_stream;
  *out = s;
  return ADG_OK;
}

adg_status adg_set_state(adg_solver *s, const double *w, int64_t count, int32_t where) {
  if (!s || !w) return ADG_ERR_ARG;
  const Layout &L = s->P.lay;
  const int VM = L.V * L.M;
  if (count != (int64_t)L.E * VM) return fail(s, ADG_ERR_ARG, "state size mismatch");
  if (where == ADG_HOST) {
    HIP_TRY(s, upload_state_host(s->P, w, s->stream));
  } else if (where == ADG_DEVICE) {
    HIP_TRY(s, launch_to_planes(w, s->P.W[0], L.E, VM, s->stream));
  } else {
    return fail(s, ADG_ERR_ARG, "where must be ADG_HOST or ADG_DEVICE");
  }
  s->cur = 0;
  s->par = 0;
  HIP_TRY(s, reset_problem(s->P, s->stream));
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
    // the graph starts from the state buffer and step counter parity it was captured
    // with; a plain step realigns them (alternating state buffers of 2N schemes and
    // limited Shu-Osher, an odd number of steps per graph) when needed
    int left = n_steps;
    while (left > 0) {
      if (left >= s->graph_steps && s->cur == s->graph_cur && s->par == s->graph_par) {
        HIP_TRY(s, hipGraphLaunch(s->gexec, s->stream));
        s->cur = s->graph_cur_after;
        s->par = s->graph_par_after;
        left -= s->graph_steps;
      } else {
        adg_status rc = enqueue_step(s, s->stream, nullptr);
        if (rc != ADG_OK) return rc;
        left -= 1;
      }
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
  HIP_TRY(s, hipMemcpy(&err, s->P.err, sizeof(int), hipMemcpyDeviceToHost));
  if (err) return fail(s, ADG_ERR_STATE, "non-physical state (rho <= 0, p <= 0, non-finite or no T convergence)");
  return ADG_OK;
}

adg_status adg_get_state(adg_solver *s, double *w, int64_t count, int32_t where) {
  if (!s || !w) return ADG_ERR_ARG;
  const Layout &L = s->P.lay;
  const int VM = L.V * L.M;
  if (count != (int64_t)L.E * VM) return fail(s, ADG_ERR_ARG, "state size mismatch");
  if (where == ADG_HOST) {
    HIP_TRY(s, download_state_host(s->P, s->P.W[s->cur], w, s->stream));
  } else if (where == ADG_DEVICE) {
    HIP_TRY(s, launch_from_planes(s->P.W[s->cur], w, L.E, VM, s->stream));
  } else {
    return fail(s, ADG_ERR_ARG, "where must be ADG_HOST or ADG_DEVICE");
  }
  return adg_sync(s);
}

adg_status adg_get_flags(adg_solver *s, int8_t *flags, int64_t *total) {
  if (!s) return ADG_ERR_ARG;
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  if (flags) HIP_TRY(s, hipMemcpy(flags, s->P.flags, (size_t)s->P.lay.E, hipMemcpyDeviceToHost));
  if (total) {
    unsigned long long c = 0;
    HIP_TRY(s, hipMemcpy(&c, s->P.flag_count, sizeof c, hipMemcpyDeviceToHost));
    *total = (int64_t)c;
  }
  return ADG_OK;
}

int64_t adg_step_count(adg_solver *s) {
  if (!s) return -1;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return -1;
  long long n = 0;
  if (hipMemcpy(&n, s->P.step + s->par, sizeof n, hipMemcpyDeviceToHost) != hipSuccess) return -1;
  return n;
}

int32_t adg_n_interfaces(const adg_solver *s) { return s ? s->P.lay.nif : -1; }

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
  for (int stage = 0; stage < s->P.lay.S; ++stage) order.push_back(0);
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

adg_status adg_autotune(adg_solver *s, int32_t n_reps, int32_t *choice) {
  if (!s || n_reps < 1) return ADG_ERR_ARG;
  if (choice) *choice = 0;
  if (s->P.phys.model != ADG_DETAILED) return ADG_OK;   // one decomposition only
  const int M = s->P.lay.M;
  // first-stage launches only: they read the state and write the first stage's output
  // buffer (and the 2N register, whose old value the first stage does not read) and the
  // level's first-stage history, all of which the next step recomputes; the state is untouched
  NsArgs a = s->P.na;
  a.rk = rk_stage(s->P.disc.rk, 0);
  const int bi = a.rk.two_n ? s->cur : 0, bo = a.rk.two_n ? (s->cur + 1) % 2 : 1;
  a.w0 = s->P.W[0];
  a.ws = s->P.W[bi];
  a.wout = s->P.W[bo];
  a.stage = 0;
  a.advance = 0;
  a.par = s->par;
  // every candidate warmed up first, then timed in three interleaved rounds; each keeps
  // its fastest round (clock ramp-up and other transients then bias no candidate)
  double t[kNsConfigs];
  hipEvent_t e0, e1;
  HIP_TRY(s, hipEventCreate(&e0));
  HIP_TRY(s, hipEventCreate(&e1));
  for (int c = 0; c < kNsConfigs; ++c) {
    for (int r = 0; r < 2; ++r) HIP_TRY(s, launch_ns_stage(M, c, a, s->stream));
    t[c] = 1e30;
  }
  for (int round = 0; round < 3; ++round)
    for (int c = 0; c < kNsConfigs; ++c) {
      HIP_TRY(s, hipEventRecord(e0, s->stream));
      for (int r = 0; r < n_reps; ++r) HIP_TRY(s, launch_ns_stage(M, c, a, s->stream));
      HIP_TRY(s, hipEventRecord(e1, s->stream));
      HIP_TRY(s, hipEventSynchronize(e1));
      float ms = 0.0f;
      HIP_TRY(s, hipEventElapsedTime(&ms, e0, e1));
      t[c] = std::min(t[c], (double)ms);
    }
  int best = 0;
  for (int c = 1; c < kNsConfigs; ++c)
    if (t[c] < t[best]) best = c;
  // the first decomposition stays unless the fastest beats it by more than 3 %: candidates
  // closer than that trade places from run to run (and under a profiler's dispatch overhead)
  if (t[best] > 0.97 * t[0]) best = 0;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best != s->ns_cfg) {
    s->ns_cfg = best;
    destroy_graph(s);
  }
  if (choice) *choice = best;
  return adg_sync(s);
}

adg_status adg_set_kernel_config(adg_solver *s, int32_t config) {
  if (!s) return ADG_ERR_ARG;
  const int n = s->P.phys.model == ADG_DETAILED ? kNsConfigs : 1;
  if (config < 0 || config >= n) return fail(s, ADG_ERR_ARG, "no such work decomposition");
  if (s->P.phys.model == ADG_DETAILED && config != s->ns_cfg) {
    s->ns_cfg = config;
    destroy_graph(s);
  }
  return ADG_OK;
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
