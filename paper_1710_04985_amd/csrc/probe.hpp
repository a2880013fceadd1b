// Hop-latency probe (probe.hip).
#pragma once

#include <hip/hip_runtime_api.h>

namespace sptrsv {

// Launch of peer+1 one-wavefront workgroups (a few, so all are resident on
// an idle GPU; were one not, its partner's bounded wait would end the
// probe); workgroups 0 and peer exchange `iters` round trips through a and b
// (device ints, zeroed by the caller).  *ticks: wall-clock ticks of rounds
// 1..iters-1 (round 0 warms up); *status set to 1 if a wait exceeded
// spin_limit polls.
hipError_t launch_pingpong(int* a, int* b, int peer, int iters, int spin_limit, long long* ticks,
                           int* status, hipStream_t s);

}  // namespace sptrsv
