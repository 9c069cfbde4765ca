// Weighted-event epilogue of the |M|^2 kernels (the unweighting step of the
// paper's Sec. 3 and Table 2, fused into the kernel that produces |M|^2).
//
// With prm.w_fac set, the lane that stores |M|^2_e also forms the event
// weight w_e = |M|^2_e * f_e (NaN and negative products clamped to 0), stores
// it when prm.w_out is set, and raises the batch maximum, held as the bit
// pattern of a non-negative double (whose integer order is the numeric
// order) in *prm.w_max, which the launch clears first.  A lane reads the
// running maximum before it competes: only a weight above it issues an
// atomic.  The product and the clamp are the ones of me_max_weight, so the
// fused and the separate forms agree bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "me_types.h"

namespace me {

__device__ __forceinline__ void store_me(const MeParams& prm, double* __restrict__ out, int64_t e, double v) {
  out[e] = v;
  if (prm.w_fac) {
    double x = v * prm.w_fac[e];
    if (!(x > 0.0)) x = 0.0;
    if (prm.w_out) prm.w_out[e] = x;
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
    if (b > __hip_atomic_load(prm.w_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(prm.w_max, b);
  }
}

// The epilogue pointers of events [e0, ...) of a launch that covers a chunk
// of the batch starting at event e0.
__host__ __forceinline__ MeParams epilogue_at(const MeParams& prm, int64_t e0) {
  MeParams c = prm;
  if (c.w_fac) {
    c.w_fac += e0;
    if (c.w_out) c.w_out += e0;
  }
  return c;
}

}  // namespace me
