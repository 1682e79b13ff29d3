// Batched ADG instances in one device workspace (the adg_batch_* C ABI).
//
// The caller's workspace holds a header (per-slot kernel argument blocks, the
// work list of the launches, per-slot step counters and error flags) followed
// by a heap from which each admitted instance takes one contiguous region
// (first fit, coalescing on release).  An admission that does not fit is
// refused with ADG_ERR_NOMEM: admission is by device-memory footprint.
//
// A time step launches, per stage, one batched kernel for all detailed-
// chemistry instances (orders dispatched inside the kernel) and one batched
// kernel per (order, flux, limiter) group of one-step instances, the limiter of
// limited instances inside that kernel.  Every workgroup works on one instance
// only, with that instance's own arguments, so the arithmetic of an instance
// does not depend on what else is in the batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "adg.h"
#include "adg_internal.hpp"
#include "adg_ns.hpp"
#include "adg_problem.hpp"

using namespace adg;

namespace {

struct Slot {
  bool used = false;
  Problem P;
  size_t off = 0, bytes = 0;  // heap region
  long long target = kNoTarget;
  int mech = -1;              // shared mechanism slot (detailed chemistry)
};

// Distinct mechanisms a batch holds at once: instances with byte-identical
// mechanisms share one device copy (all the tiles of a batch of one mechanism
// then read the same few kilobytes, which stay in every L2).
constexpr int kBatchMechs = 16;

constexpr int kGroupStreams = 4;

struct Group {
  int kind;  // 0 detailed stage, 1 one-step stage
  int M, flux;
  bool lim;  // one-step instances with the limiter (in the stage kernel)
  int off, n;  // range of the work list
};


}  // namespace

struct adg_batch {
  hipStream_t stream = nullptr;
  int precision = ADG_FP64;
  char *ws = nullptr;
  size_t bytes = 0;
  int max_inst = 0;
  long long max_elem = 0;
  long long max_tiles = 0;
  NsArgs *d_ns = nullptr;
  EulerSet *d_eu = nullptr;
  NsMech *d_mech = nullptr;
  std::vector<NsMech> mech_host = std::vector<NsMech>(kBatchMechs);
  std::vector<int> mech_ref = std::vector<int>(kBatchMechs, 0);
  int2 *d_tiles = nullptr;
  long long *d_step = nullptr;   // [slot][2]: each instance's step counters of the two parities
  int *d_err = nullptr;
  int par = 0;                   // step counter parity of the next batch step
  size_t heap_off = 0;
  std::map<size_t, size_t> free_list;  // offset -> bytes
  std::vector<Slot> slots;
  long long elems = 0;
  int active = 0;
  bool dirty = true;
  int tile_elems = 8;        // elements per tile of the detailed-chemistry kernel (4 or 8)
  std::vector<Group> groups;
  std::vector<int2> h_tiles;
  int graph_steps = 0;
  bool graph_valid = false;
  // graph p replays graph_steps steps from step counter parity p (launch arguments of the
  // batched kernels), so a replay never waits for a realigning plain step
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;
  // launches of a stage's groups spread over the batch's stream and up to kGroupStreams - 1
  // extra streams (default priority), joined before the next stage; 1 = all on one stream
  int group_streams = kGroupStreams;
  hipStream_t aux[kGroupStreams - 1] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kGroupStreams - 1] = {};
  std::vector<hipEvent_t> prof_events;
  std::vector<int> prof_class;
  std::string msg;
};

namespace {

struct Header {
  size_t ns, eu, mech, tiles, step, err, total;
};

Header header_layout(int max_inst, long long max_tiles) {
  Header h;
  size_t off = 0;
  h.ns = off;    off += align256(sizeof(NsArgs) * (size_t)max_inst);
  h.eu = off;    off += align256(sizeof(EulerSet) * (size_t)max_inst);
  h.mech = off;  off += align256(sizeof(NsMech) * (size_t)kBatchMechs);
  h.tiles = off; off += align256(sizeof(int2) * (size_t)max_tiles);
  h.step = off;  off += align256(2 * sizeof(long long) * (size_t)max_inst);
  h.err = off;   off += align256(sizeof(int) * (size_t)max_inst);
  h.total = off;
  return h;
}

long long tile_bound(int max_inst, long long max_elem) {
  return (max_elem + kNsMinTile - 1) / kNsMinTile + 4LL * max_inst;
}

adg_status bfail(adg_batch *b, adg_status code, const std::string &m) {
  if (b) b->msg = m;
  return code;
}

#define BHIP(b, expr)                                                                    \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) return bfail(b, ADG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

bool heap_take(adg_batch *b, size_t need, size_t &off) {
  for (auto it = b->free_list.begin(); it != b->free_list.end(); ++it) {
    if (it->second >= need) {
      off = it->first;
      const size_t rest = it->second - need;
      b->free_list.erase(it);
      if (rest) b->free_list[off + need] = rest;
      return true;
    }
  }
  return false;
}

void heap_give(adg_batch *b, size_t off, size_t bytes) {
  auto it = b->free_list.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != b->free_list.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    b->free_list.erase(nx);
  }
  if (it != b->free_list.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      b->free_list.erase(it);
    }
  }
}

// Work list: detailed instances first (one group), then one-step instances by
// (order, flux, limiter).  Entries of one instance are consecutive.
void rebuild_tiles(adg_batch *b) {
  b->groups.clear();
  b->h_tiles.clear();
  auto add_group = [&](int kind, int M, int flux, bool lim, auto pick, auto nblocks) {
    Group g{kind, M, flux, lim, (int)b->h_tiles.size(), 0};
    for (int i = 0; i < (int)b->slots.size(); ++i) {
      const Slot &s = b->slots[i];
      if (!s.used || !pick(s)) continue;
      const int nb = nblocks(s);
      for (int k = 0; k < nb; ++k) b->h_tiles.push_back(make_int2(i, k * (kind == 0 ? b->tile_elems : 1)));
    }
    g.n = (int)b->h_tiles.size() - g.off;
    // XCD-aware order: workgroup p of the launch takes work item xcd_item(p, n), so each XCD
    // works through a contiguous run of tiles (same instances, shared halos, one L2)
    std::vector<int2> run(b->h_tiles.begin() + g.off, b->h_tiles.end());
    for (int p = 0; p < g.n; ++p) b->h_tiles[g.off + p] = run[xcd_item(p, g.n)];
    if (g.n > 0) b->groups.push_back(g);
  };
  add_group(0, 0, 0, false, [](const Slot &s) { return s.P.phys.model == ADG_DETAILED; },
            [&](const Slot &s) { return (s.P.lay.E + b->tile_elems - 1) / b->tile_elems; });
  if (!b->groups.empty() && b->groups[0].kind == 0) {
    int mm = 2;
    for (const Slot &s : b->slots)
      if (s.used && s.P.phys.model == ADG_DETAILED) mm = std::max(mm, s.P.lay.M);
    b->groups[0].M = mm;
  }
  for (int M = 2; M <= kMaxM; ++M)
    for (int flux = 0; flux <= 1; ++flux)
      for (int lim = 0; lim <= 1; ++lim)
        add_group(1, M, flux, lim != 0,
                  [&](const Slot &s) {
                    return s.P.phys.model == ADG_ONESTEP && s.P.lay.M == M && s.P.disc.flux == flux &&
                           (s.P.disc.limiter != 0) == (lim != 0);
                  },
                  [&](const Slot &s) { return euler_blocks(s.P.lay.E, lim != 0); });
}

// The extra streams and events of concurrent group launches, created on first use.
adg_status ensure_group_streams(adg_batch *b) {
  if (b->fork) return ADG_OK;
  for (int k = 0; k < kGroupStreams - 1; ++k) {
    BHIP(b, hipStreamCreateWithFlags(&b->aux[k], hipStreamNonBlocking));
    BHIP(b, hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming));
  }
  BHIP(b, hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  return ADG_OK;
}

adg_status enqueue_batch_step(adg_batch *b, hipStream_t st, bool timed) {
  // a stage's groups touch disjoint instances: with several groups they may run side by side
  // (group k on stream k mod S, the first on st), every stream joined back before the next stage
  const int nstreams = timed ? 1 : std::min<int>(b->group_streams, (int)b->groups.size());
  if (nstreams > 1) {
    adg_status rc = ensure_group_streams(b);
    if (rc != ADG_OK) return rc;
  }
  for (int stage = 0; stage < 3; ++stage) {
    if (nstreams > 1) {
      BHIP(b, hipEventRecord(b->fork, st));
      for (int k = 1; k < nstreams; ++k) BHIP(b, hipStreamWaitEvent(b->aux[k - 1], b->fork, 0));
    }
    for (int gi = 0; gi < (int)b->groups.size(); ++gi) {
      const Group &g = b->groups[gi];
      const hipStream_t gs = nstreams > 1 && gi % nstreams ? b->aux[gi % nstreams - 1] : st;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (timed) {
        BHIP(b, hipEventCreate(&e0));
        BHIP(b, hipEventRecord(e0, st));
      }
      if (g.kind == 0) {
        BHIP(b, launch_ns_batch(b->d_ns, b->d_tiles + g.off, g.n, stage, b->par, b->precision == ADG_MIXED_FP32,
                                g.M, b->tile_elems, gs));
      } else {
        BHIP(b, launch_euler_batch(g.M, g.flux, g.lim, b->d_eu, b->d_tiles + g.off, g.n, stage, b->par, gs));
      }
      if (timed) {
        BHIP(b, hipEventCreate(&e1));
        BHIP(b, hipEventRecord(e1, st));
        b->prof_events.push_back(e0);
        b->prof_events.push_back(e1);
        b->prof_class.push_back(g.kind);
      }
    }
    if (nstreams > 1) {
      for (int k = 1; k < nstreams; ++k) {
        BHIP(b, hipEventRecord(b->join[k - 1], b->aux[k - 1]));
        BHIP(b, hipStreamWaitEvent(st, b->join[k - 1], 0));
      }
    }
  }
  b->par ^= 1;   // the step's last launches wrote the next counts into the other counters
  return ADG_OK;
}

void destroy_batch_graph(adg_batch *b) {
  for (int p = 0; p < 2; ++p) {
    if (b->gexec[p]) (void)hipGraphExecDestroy(b->gexec[p]);
    if (b->graph[p]) (void)hipGraphDestroy(b->graph[p]);
    b->gexec[p] = nullptr;
    b->graph[p] = nullptr;
  }
  b->graph_valid = false;
}

adg_status prepare(adg_batch *b) {
  if (!b->dirty) return ADG_OK;
  destroy_batch_graph(b);
  rebuild_tiles(b);
  if ((long long)b->h_tiles.size() > b->max_tiles) return bfail(b, ADG_ERR_NOMEM, "work list exceeds its capacity");
  BHIP(b, hipStreamSynchronize(b->stream));
  if (!b->h_tiles.empty())
    BHIP(b, hipMemcpy(b->d_tiles, b->h_tiles.data(), sizeof(int2) * b->h_tiles.size(), hipMemcpyHostToDevice));
  b->dirty = false;
  return ADG_OK;
}

adg_status build_batch_graph(adg_batch *b) {
  destroy_batch_graph(b);
  if (!b->cap_stream) BHIP(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  const int par_keep = b->par;
  for (int p = 0; p < 2; ++p) {
    b->par = p;
    BHIP(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    adg_status rc = ADG_OK;
    for (int i = 0; i < b->graph_steps && rc == ADG_OK; ++i) rc = enqueue_batch_step(b, b->cap_stream, false);
    b->par = par_keep;   // nothing ran: capture only records
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc != ADG_OK) {
      if (g) (void)hipGraphDestroy(g);
      destroy_batch_graph(b);
      return rc;
    }
    if (e != hipSuccess) {
      destroy_batch_graph(b);
      return bfail(b, ADG_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    b->graph[p] = g;
    e = hipGraphInstantiate(&b->gexec[p], g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      destroy_batch_graph(b);
      return bfail(b, ADG_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
  }
  b->graph_valid = true;
  return ADG_OK;
}

bool valid_slot(const adg_batch *b, int slot) { return b && slot >= 0 && slot < b->max_inst && b->slots[slot].used; }

}  // namespace

extern "C" {

size_t adg_batch_header_bytes(int32_t max_instances, int64_t max_elements) {
  if (max_instances < 1 || max_elements < 1) return 0;
  return header_layout(max_instances, tile_bound(max_instances, max_elements)).total;
}

size_t adg_batch_instance_bytes(const adg_physics *phys, const adg_discretization *disc, const adg_async *as) {
  Layout L;
  if (!make_layout(phys, disc, as, L, nullptr, true)) return 0;
  return align256(L.total);
}

adg_status adg_batch_create(int32_t max_instances, int64_t max_elements, int32_t precision, void *device_workspace,
                            size_t workspace_bytes, void *hip_stream, adg_batch **out) {
  if (!out) return ADG_ERR_ARG;
  *out = nullptr;
  if (max_instances < 1 || max_elements < 1) return ADG_ERR_ARG;
  if (precision == ADG_MIXED_BF16) return ADG_ERR_UNSUPPORTED;   // beyond the error budget (adg.h)
  if (precision != ADG_FP64 && precision != ADG_MIXED_FP32) return ADG_ERR_ARG;
  if (!device_workspace || ((uintptr_t)device_workspace & 255)) return ADG_ERR_ARG;
  const long long max_tiles = tile_bound(max_instances, max_elements);
  if (max_tiles > 0x7fffffffLL) return ADG_ERR_ARG;
  const Header h = header_layout(max_instances, max_tiles);
  if (workspace_bytes < h.total) return ADG_ERR_NOMEM;
  adg_batch *b = new adg_batch();
  b->stream = (hipStream_t)hip_stream;
  b->precision = precision;
  b->ws = (char *)device_workspace;
  b->bytes = workspace_bytes;
  b->max_inst = max_instances;
  b->max_elem = max_elements;
  b->max_tiles = max_tiles;
  b->d_ns = (NsArgs *)(b->ws + h.ns);
  b->d_eu = (EulerSet *)(b->ws + h.eu);
  b->d_mech = (NsMech *)(b->ws + h.mech);
  b->d_tiles = (int2 *)(b->ws + h.tiles);
  b->d_step = (long long *)(b->ws + h.step);
  b->d_err = (int *)(b->ws + h.err);
  b->heap_off = h.total;
  const size_t heap = (workspace_bytes - h.total) & ~(size_t)255;
  if (heap) b->free_list[h.total] = heap;
  b->slots.resize(max_instances);
  *out = b;
  return ADG_OK;
}

adg_status adg_batch_add(adg_batch *b, const adg_physics *phys, const adg_discretization *disc, const adg_async *as,
                         const double *w0, int64_t count, int32_t where, int64_t n_steps, int32_t *slot_out) {
  if (!b || !w0 || !slot_out || n_steps < 0) return ADG_ERR_ARG;
  *slot_out = -1;
  Layout L;
  std::string why;
  if (!make_layout(phys, disc, as, L, &why, true)) return bfail(b, ADG_ERR_ARG, why);
  if (count != (int64_t)L.E * L.V * L.M) return bfail(b, ADG_ERR_ARG, "state size mismatch");
  if (where != ADG_HOST && where != ADG_DEVICE) return bfail(b, ADG_ERR_ARG, "where must be ADG_HOST or ADG_DEVICE");
  if (disc->rk != ADG_SSPRK3) return bfail(b, ADG_ERR_UNSUPPORTED, "batches run SSP-RK3 only");
  if (disc->precision == ADG_MIXED_BF16) return bfail(b, ADG_ERR_UNSUPPORTED, "ADG_MIXED_BF16 is not supported");
  if (disc->precision != ADG_FP64 && disc->precision != b->precision)
    return bfail(b, ADG_ERR_ARG, "instance precision differs from the batch's");
  if (phys->model == ADG_DETAILED && phys->n_species > kNsMaxSpecies)
    return bfail(b, ADG_ERR_UNSUPPORTED, "batched detailed-chemistry instances take up to 9 species");
  if (phys->model == ADG_DETAILED && phys->mech && phys->mech->n_reactions > kNsBatchReactions)
    return bfail(b, ADG_ERR_UNSUPPORTED, "batched detailed-chemistry instances take up to 24 reactions");
  int slot = -1;
  for (int i = 0; i < b->max_inst; ++i)
    if (!b->slots[i].used) { slot = i; break; }
  if (slot < 0) return bfail(b, ADG_ERR_NOMEM, "no free instance slot");
  if (b->elems + L.E > b->max_elem) return bfail(b, ADG_ERR_NOMEM, "element capacity of the batch exceeded");
  const size_t need = align256(L.total);
  size_t off = 0;
  if (!heap_take(b, need, off)) return bfail(b, ADG_ERR_NOMEM, "no free workspace region large enough");
  // kernels still in flight may read the region that was just handed out
  hipError_t he = hipStreamSynchronize(b->stream);
  Slot s;
  adg_status rc = he == hipSuccess ? setup_problem(phys, disc, as, b->ws + off, L, s.P) : ADG_ERR_HIP;
  if (rc != ADG_OK) {
    heap_give(b, off, need);
    return bfail(b, rc, rc == ADG_ERR_HIP ? "HIP call failed while placing the instance" : "unsupported instance");
  }
  s.used = true;
  s.off = off;
  s.bytes = need;
  s.target = n_steps > 0 ? n_steps : kNoTarget;
  // counters of the slot live in the header so that one copy reads them all
  Problem &P = s.P;
  P.step = b->d_step + 2 * (size_t)slot;
  P.err = b->d_err + slot;
  auto fail_release = [&](hipError_t e, const char *what) {
    heap_give(b, off, need);
    return bfail(b, ADG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  if (P.phys.model == ADG_DETAILED) {
    NsMech hm;
    if (ns_build_mech(phys, hm) != ADG_OK) {
      heap_give(b, off, need);
      return bfail(b, ADG_ERR_UNSUPPORTED, "unsupported mechanism");
    }
    int ms = -1;
    for (int j = 0; j < kBatchMechs && ms < 0; ++j)
      if (b->mech_ref[j] > 0 && std::memcmp(&b->mech_host[j], &hm, sizeof hm) == 0) ms = j;
    if (ms < 0) {
      for (int j = 0; j < kBatchMechs && ms < 0; ++j)
        if (b->mech_ref[j] == 0) ms = j;
      if (ms < 0) {
        heap_give(b, off, need);
        return bfail(b, ADG_ERR_NOMEM, "too many distinct mechanisms in the batch");
      }
      he = hipMemcpy(b->d_mech + ms, &hm, sizeof hm, hipMemcpyHostToDevice);
      if (he != hipSuccess) return fail_release(he, "mechanism upload");
      b->mech_host[ms] = hm;
    }
    s.mech = ms;
    NsArgs na = P.na;
    na.mech = b->d_mech + ms;
    na.step = P.step;
    na.err = P.err;
    na.target = s.target;
    he = hipMemcpy(b->d_ns + slot, &na, sizeof na, hipMemcpyHostToDevice);
    if (he != hipSuccess) return fail_release(he, "descriptor upload");
  } else {
    EulerSet es;
    std::memset(&es, 0, sizeof es);
    const int in_buf[3] = {0, 1, 2}, out_buf[3] = {1, 2, 0};
    for (int st = 0; st < 3; ++st) {
      EulerArgs a = P.ea;   // with the limiter a.alt is set: the kernel picks the buffers
      a.w0 = P.W[0];
      a.ws = P.W[in_buf[st]];
      a.wout = P.W[out_buf[st]];
      a.stage = st;
      a.rk = rk_stage(ADG_SSPRK3, st);
      a.advance = st == 2;
      a.step = P.step;
      a.err = P.err;
      a.target = s.target;
      es.st[st] = a;
    }
    if (P.disc.limiter) es.lim = P.la;
    he = hipMemcpy(b->d_eu + slot, &es, sizeof es, hipMemcpyHostToDevice);
    if (he != hipSuccess) return fail_release(he, "descriptor upload");
  }
  const int VM = L.V * L.M;
  if (where == ADG_HOST) he = upload_state_host(P, w0, b->stream);
  else he = launch_to_planes(w0, P.W[0], L.E, VM, b->stream);
  if (he == hipSuccess) he = reset_problem(P, b->stream);
  if (he == hipSuccess) he = launch_zero(P.step, 2 * sizeof(long long), b->stream);
  if (he == hipSuccess) he = launch_zero(P.err, sizeof(int), b->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(b->stream);
  if (he != hipSuccess) return fail_release(he, "initial state");
  b->slots[slot] = s;
  if (s.mech >= 0) b->mech_ref[s.mech] += 1;
  b->elems += L.E;
  b->active += 1;
  b->dirty = true;
  *slot_out = slot;
  return ADG_OK;
}

adg_status adg_batch_remove(adg_batch *b, int32_t slot) {
  if (!valid_slot(b, slot)) return bfail(b, ADG_ERR_ARG, "no instance in this slot");
  BHIP(b, hipStreamSynchronize(b->stream));
  Slot &s = b->slots[slot];
  heap_give(b, s.off, s.bytes);
  if (s.mech >= 0) b->mech_ref[s.mech] -= 1;
  b->elems -= s.P.lay.E;
  b->active -= 1;
  s = Slot();
  b->dirty = true;
  return ADG_OK;
}

adg_status adg_batch_step(adg_batch *b, int32_t n_steps) {
  if (!b || n_steps < 0) return ADG_ERR_ARG;
  adg_status rc = prepare(b);
  if (rc != ADG_OK) return rc;
  if (b->groups.empty()) return ADG_OK;
  int done = 0;
  if (b->graph_steps > 0) {
    if (!b->graph_valid) {
      rc = build_batch_graph(b);
      if (rc != ADG_OK) return rc;
    }
    // whole graphs from the graph of the current parity, then plain steps for the rest
    while (done + b->graph_steps <= n_steps) {
      BHIP(b, hipGraphLaunch(b->gexec[b->par], b->stream));
      b->par ^= b->graph_steps & 1;
      done += b->graph_steps;
    }
  }
  for (; done < n_steps; ++done) {
    rc = enqueue_batch_step(b, b->stream, false);
    if (rc != ADG_OK) return rc;
  }
  return ADG_OK;
}

adg_status adg_batch_poll(adg_batch *b, int64_t *steps, int32_t *state_err) {
  if (!b) return ADG_ERR_ARG;
  BHIP(b, hipStreamSynchronize(b->stream));
  std::vector<long long> st(2 * (size_t)b->max_inst);
  std::vector<int> er(b->max_inst);
  BHIP(b, hipMemcpy(st.data(), b->d_step, 2 * sizeof(long long) * b->max_inst, hipMemcpyDeviceToHost));
  BHIP(b, hipMemcpy(er.data(), b->d_err, sizeof(int) * b->max_inst, hipMemcpyDeviceToHost));
  for (int i = 0; i < b->max_inst; ++i) {
    const bool u = b->slots[i].used;
    if (steps) steps[i] = u ? st[2 * (size_t)i + b->par] : -1;
    if (state_err) state_err[i] = u ? (er[i] != 0) : 0;
  }
  return ADG_OK;
}

adg_status adg_batch_get_state(adg_batch *b, int32_t slot, double *w, int64_t count, int32_t where) {
  if (!valid_slot(b, slot) || !w) return bfail(b, ADG_ERR_ARG, "no instance in this slot");
  const Problem &P = b->slots[slot].P;
  const Layout &L = P.lay;
  const int VM = L.V * L.M;
  if (count != (int64_t)L.E * VM) return bfail(b, ADG_ERR_ARG, "state size mismatch");
  // with the limiter the state lives in buffer (step count) mod 2
  const double *src = P.W[0];
  if (P.ea.alt) {
    long long n = 0;
    BHIP(b, hipStreamSynchronize(b->stream));
    BHIP(b, hipMemcpy(&n, P.step + b->par, sizeof n, hipMemcpyDeviceToHost));
    src = P.W[n & 1];
  }
  if (where == ADG_HOST) {
    BHIP(b, download_state_host(P, src, w, b->stream));
  } else if (where == ADG_DEVICE) {
    BHIP(b, launch_from_planes(src, w, L.E, VM, b->stream));
  } else {
    return bfail(b, ADG_ERR_ARG, "where must be ADG_HOST or ADG_DEVICE");
  }
  BHIP(b, hipStreamSynchronize(b->stream));
  int err = 0;
  BHIP(b, hipMemcpy(&err, P.err, sizeof err, hipMemcpyDeviceToHost));
  if (err) return bfail(b, ADG_ERR_STATE, "non-physical state in this instance");
  return ADG_OK;
}

adg_status adg_batch_set_graph(adg_batch *b, int32_t steps_per_graph) {
  if (!b || steps_per_graph < 0) return ADG_ERR_ARG;
  if (steps_per_graph != b->graph_steps) destroy_batch_graph(b);
  b->graph_steps = steps_per_graph;
  return ADG_OK;
}

adg_status adg_batch_profile(adg_batch *b, int32_t n_steps, double *ms_out, int64_t *launches_out, int32_t n_classes) {
  if (!b || n_steps < 1 || !ms_out || !launches_out || n_classes < 1) return ADG_ERR_ARG;
  adg_status rc = prepare(b);
  if (rc != ADG_OK) return rc;
  b->prof_events.clear();
  b->prof_class.clear();
  for (int i = 0; i < n_steps && rc == ADG_OK; ++i) rc = enqueue_batch_step(b, b->stream, true);
  hipError_t he = hipStreamSynchronize(b->stream);
  std::vector<double> sum(n_classes, 0.0);
  std::vector<int64_t> cnt(n_classes, 0);
  for (size_t k = 0; k < b->prof_class.size(); ++k) {
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, b->prof_events[2 * k], b->prof_events[2 * k + 1]);
    const int c = b->prof_class[k];
    if (c < n_classes) { sum[c] += ms; cnt[c] += 1; }
  }
  for (hipEvent_t ev : b->prof_events) (void)hipEventDestroy(ev);
  b->prof_events.clear();
  b->prof_class.clear();
  if (rc != ADG_OK) return rc;
  if (he != hipSuccess) return bfail(b, ADG_ERR_HIP, hipGetErrorString(he));
  for (int c = 0; c < n_classes; ++c) {
    ms_out[c] = cnt[c] ? sum[c] / cnt[c] : 0.0;
    launches_out[c] = cnt[c];
  }
  return ADG_OK;
}

adg_status adg_batch_autotune(adg_batch *b, int32_t n_reps, int32_t *choice) {
  if (!b || n_reps < 1) return ADG_ERR_ARG;
  static const int kTiles[2] = {8, 4};
  double t[2] = {1e30, 1e30};
  bool any = false;
  // both candidates timed in three interleaved rounds, each keeping its fastest round
  for (int round = 0; round < 3; ++round) {
    for (int c = 0; c < 2; ++c) {
      b->tile_elems = kTiles[c];
      b->dirty = true;
      adg_status rc = prepare(b);
      if (rc != ADG_OK) return rc;
      const Group *g = nullptr;
      for (const Group &x : b->groups)
        if (x.kind == 0) g = &x;
      if (!g) break;   // no detailed-chemistry instance: nothing to choose
      any = true;
      // stage-0 launches only: they read w^n and write the first stage buffer and the
      // level's stage-0 history, which the next step recomputes; the state is untouched
      hipEvent_t e0, e1;
      BHIP(b, hipEventCreate(&e0));
      BHIP(b, hipEventCreate(&e1));
      BHIP(b, launch_ns_batch(b->d_ns, b->d_tiles + g->off, g->n, 0, b->par, b->precision == ADG_MIXED_FP32, g->M,
                              b->tile_elems, b->stream));   // warm-up
      BHIP(b, hipEventRecord(e0, b->stream));
      for (int r = 0; r < n_reps; ++r)
        BHIP(b, launch_ns_batch(b->d_ns, b->d_tiles + g->off, g->n, 0, b->par, b->precision == ADG_MIXED_FP32, g->M,
                                b->tile_elems, b->stream));
      BHIP(b, hipEventRecord(e1, b->stream));
      BHIP(b, hipEventSynchronize(e1));
      float ms = 0.0f;
      BHIP(b, hipEventElapsedTime(&ms, e0, e1));
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      t[c] = std::min(t[c], (double)ms);
    }
    if (!any) break;
  }
  const int best = any && t[1] < t[0] ? 1 : 0;
  b->tile_elems = kTiles[best];
  b->dirty = true;
  if (choice) *choice = best;
  return prepare(b);
}

adg_status adg_batch_set_kernel_config(adg_batch *b, int32_t config) {
  if (!b) return ADG_ERR_ARG;
  if (config < 0 || config > 1) return bfail(b, ADG_ERR_ARG, "no such work decomposition");
  b->tile_elems = config ? 4 : 8;
  b->dirty = true;
  return ADG_OK;
}

int32_t adg_batch_active(const adg_batch *b) { return b ? b->active : -1; }

int64_t adg_batch_free_bytes(const adg_batch *b) {
  if (!b) return -1;
  size_t best = 0;
  for (const auto &kv : b->free_list) best = std::max(best, kv.second);
  return (int64_t)best;
}

void adg_batch_destroy(adg_batch *b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  destroy_batch_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (int k = 0; k < kGroupStreams - 1; ++k) {
    if (b->aux[k]) {
      (void)hipStreamSynchronize(b->aux[k]);
      (void)hipStreamDestroy(b->aux[k]);
    }
    if (b->join[k]) (void)hipEventDestroy(b->join[k]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
}

adg_status adg_batch_set_group_streams(adg_batch *b, int32_t streams) {
  if (!b) return ADG_ERR_ARG;
  if (streams < 1 || streams > kGroupStreams) return bfail(b, ADG_ERR_ARG, "group streams out of range");
  if (streams != b->group_streams) {
    b->group_streams = streams;
    destroy_batch_graph(b);   // captured with the old spread
  }
  return ADG_OK;
}

const char *adg_batch_last_error(const adg_batch *b) { return b ? b->msg.c_str() : "null batch"; }

}  // extern "C"
