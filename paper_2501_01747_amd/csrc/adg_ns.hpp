// Detailed-chemistry Navier-Stokes stage kernel: declarations.
#pragma once

#include "adg.h"
#include "adg_internal.hpp"

namespace adg {

struct NsMech {
  int dummy;
};

struct NsArgs {
  const double *w0;
  const double *ws;
  double *wout;
  int stage;
};

inline bool ns_supported(int, int) { return false; }
inline adg_status ns_setup(NsArgs &, const adg_physics *, const adg_discretization *, int, int, bool, double,
                           const DelayParams &, const RingParams &, const Tables &, const int *, const long long *,
                           int *, NsMech *) {
  return ADG_ERR_UNSUPPORTED;
}
inline hipError_t launch_ns_stage(int, const NsArgs &, hipStream_t) { return hipErrorInvalidValue; }

}  // namespace adg
