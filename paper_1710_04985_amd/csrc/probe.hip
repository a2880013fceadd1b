// Hop-latency probe: the time for a value published by one wavefront (one
// agent-scope atomic store) to be seen by a wavefront polling it on another
// CU (agent-scope atomic loads), the unit step of the self-scheduled solves'
// critical path (Sec. 4.2: a row starts once its dependencies are done).
#include <hip/hip_runtime.h>

#include "probe.hpp"

namespace sptrsv {
namespace {

// Workgroups 0 and `peer` (one wavefront each) bounce a counter: workgroup 0
// writes 1, 3, 5, ... into a, the peer answers 2, 4, 6, ... into b.  Every
// wait is bounded; a timeout sets *status and ends the exchange.  Other
// workgroups of the grid only pad the dispatch so that `peer` lands on the
// intended XCD (consecutive workgroups go to consecutive XCDs).
__global__ void __launch_bounds__(64)
k_pingpong(int* a, int* b, int peer, int iters, int spin_limit, long long* ticks, int* status) {
  const int wg = blockIdx.x;
  if ((wg != 0 && wg != peer) || threadIdx.x != 0) return;
  const bool first = wg == 0;
  int* mine = first ? a : b;
  int* theirs = first ? b : a;
  long long t0 = 0;
  for (int k = 0; k < iters; ++k) {
    const int send = 2 * k + (first ? 1 : 2);
    const int want = first ? 2 * k + 2 : 2 * k + 1;
    if (first) {
      if (k == 1) t0 = wall_clock64();   // round 0 warms the lines
      __hip_atomic_store(mine, send, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    int spins = 0;
    while (__hip_atomic_load(theirs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
      if (++spins > spin_limit) {
        __hip_atomic_store(status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
      }
    }
    if (!first) __hip_atomic_store(mine, send, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (first) *ticks = wall_clock64() - t0;
}

}  // namespace

hipError_t launch_pingpong(int* a, int* b, int peer, int iters, int spin_limit, long long* ticks,
                           int* status, hipStream_t s) {
  int grid = peer + 1;
  void* args[] = {&a, &b, &peer, &iters, &spin_limit, &ticks, &status};
  return hipLaunchKernel(reinterpret_cast<const void*>(k_pingpong), dim3(grid), dim3(64), args, 0,
                         s);
}

}  // namespace sptrsv
