// Residency check of the persistent-grid (static-schedule) kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace sptrsv {

// A static schedule (chunk lists fixed per wavefront before the launch) is
// only guaranteed to progress when every wavefront of the grid is resident:
// a waiting wavefront may wait for a chunk of any other.  Each wavefront
// signs in on `arrive` (zeroed before the launch) and waits, for at most
// `limit` polls, until the whole grid has signed in.  If it never fills,
// kStatusNotResident (and kStatusTimeout, so that every wait ends) is
// raised and the wavefront leaves; a wavefront arriving after that leaves
// too.  Returns false when the calling wavefront must leave.  limit = 0
// fails at once unless the wavefront is the last to arrive (used by tests to
// force the failure from the host).
__device__ __forceinline__ bool grid_resident(int* arrive, int limit, int* status) {
  const int expect = static_cast<int>(gridDim.x * (blockDim.x >> 6));
  int ok = 1;
  if ((threadIdx.x & 63) == 0) {
    const int me = __hip_atomic_fetch_add(arrive, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (me + 1 < expect) {
      for (int s = 0;; ++s) {
        if (s >= limit ||
            (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
             kStatusNotResident)) {
          __hip_atomic_fetch_or(status, kStatusNotResident | kStatusTimeout, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        if (__hip_atomic_load(arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= expect) break;
        __builtin_amdgcn_s_sleep(2);
      }
    }
    if (ok && (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
               kStatusNotResident))
      ok = 0;
  }
  return __builtin_amdgcn_readfirstlane(ok) != 0;
}

}  // namespace sptrsv
