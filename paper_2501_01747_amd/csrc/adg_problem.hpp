// One ADG problem placed in device memory: layout of its region of a
// workspace, device pointers and the argument blocks of its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "adg.h"
#include "adg_internal.hpp"
#include "adg_ns.hpp"

namespace adg {

constexpr long long kNoTarget = 0x7fffffffffffffffLL;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t state, flags, face_if, counters, ring, sched, mech, at, total;
  int nbuf;             // state-sized buffers (3; 4 for a 2N scheme with the limiter)
  int nif, nfaces, D, rec, q, V, M, E;
  int S;                // RK stages per step
  int off_F, off_Wc, off_U;
  bool carry_at;        // AT combinations carried between launches (single detailed problems with PE interfaces)
};

struct Problem {
  adg_physics phys{};
  adg_discretization disc{};
  adg_async as{};
  Layout lay{};
  char *base = nullptr;
  double *W[4] = {nullptr, nullptr, nullptr, nullptr};
  int8_t *flags = nullptr;
  int *face_if = nullptr;
  long long *step = nullptr;   // [2]: the step counters of the two parities
  int *err = nullptr;
  unsigned long long *flag_count = nullptr;
  double *ring = nullptr;
  double *at = nullptr;        // detailed model with PE interfaces: two per-face AT buffers
  size_t at_stride = 0;        // doubles per buffer
  EulerArgs ea{};
  LimiterArgs la{};
  NsArgs na{};
};

// Validates a problem and computes the layout of its device region (bytes in L.total).
// batched: the layout of a batch instance (no AT carry buffers: the batched kernel gathers).
bool make_layout(const adg_physics *ph, const adg_discretization *d, const adg_async *as, Layout &L,
                 std::string *why, bool batched = false);
// ADG_ERR_UNSUPPORTED for precisions a single problem cannot run (MIXED_BF16; MIXED_FP32 with
// the one-step model), with the reason in *why.
adg_status check_precision(const adg_physics *ph, const adg_discretization *d, std::string *why);
// Places the problem at `base` (256-byte aligned, L.total bytes), uploads its
// constant data and fills the kernel arguments.
adg_status setup_problem(const adg_physics *phys, const adg_discretization *disc, const adg_async *as, char *base,
                         const Layout &L, Problem &P);
hipError_t upload_state_host(const Problem &P, const double *w, hipStream_t st);
hipError_t download_state_host(const Problem &P, const double *buf, double *w, hipStream_t st);
// Step counter, error flag, history ring and flags back to zero.
hipError_t reset_problem(const Problem &P, hipStream_t st);
// Zero `bytes` bytes at p with a fill kernel on stream st (capturable, unlike hipMemsetAsync).
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);

}  // namespace adg
