// Column-wise solves (Sec. 3.2 sweep; Sec. 4.1 LEVC and Sec. 4.2 SLFC of
// Li, arXiv:1710.04985): once x_k is final, its column pushes -T(i,k) x_k into
// the accumulators of the rows i that depend on it.  Launchers are
// host-callable and enqueue on `stream`.
#pragma once

#include <hip/hip_runtime_api.h>
#include <cstdint>

#include "kernels.hpp"

namespace sptrsv {

// Push lists of one level-ordered plan: for the column solved at position k,
// entries [ptr[k], ptr[k+1]) name the positions dst[] that depend on it and
// the matrix values val[] of those dependencies (gathered from the plan's
// off-diagonal copy through src[]).
struct DevPush {
  int64_t nnz = 0;
  int* ptr = nullptr;    // [n+1]
  int* dst = nullptr;    // [nnz] dependent position
  int* src = nullptr;    // [nnz] index into the plan's off-diagonal values
  void* val = nullptr;   // [nnz] T
};

struct ColumnArgs {
  const DevPlan* plan;       // positions, diagonal, in-degrees (off_ptr)
  const DevPush* push;
  const DevChunks* chunks;   // chunks over positions, sized by push-list length
  const void* b;             // caller's right-hand side
  void* x;                   // caller's solution
  void* acc;                 // [n] T, position order: b minus the pushed updates
  int* cnt;                  // [n] updates received per position
  int* status;
  int* arrive = nullptr;     // residency check of the persistent grid
  int spin_limit = 1 << 22;
  int res_limit = 1 << 20;
  int coop = 0;              // 1 = cooperative launch, 0 = ordinary launch
  int grid = 0;
  int wg = 64;
  const int* wave_ptr = nullptr;    // self-scheduled: per-wavefront chunk lists
  const int* wave_list = nullptr;
};

// push values := the plan's off-diagonal values through push.src
template <typename T> hipError_t launch_push_gather(const DevPlan& p, const DevPush& q,
                                                    hipStream_t s);
// acc := b in position order, cnt := 0 (start of every column solve)
template <typename T> hipError_t launch_column_init(const ColumnArgs& a, hipStream_t s);
// level-scheduled (LEVC): the chunks [chunk_begin, chunk_end) of one level
template <typename T> hipError_t launch_column_level(const ColumnArgs& a, int chunk_begin,
                                                     int chunk_end, hipStream_t s);
// self-scheduled (SLFC): one persistent launch of a.grid workgroups over
// the per-wavefront chunk lists (cooperative if a.coop)
template <typename T> hipError_t launch_column_self(const ColumnArgs& a, hipStream_t s);
template <typename T> int column_self_blocks_per_cu(int wg);

}  // namespace sptrsv
