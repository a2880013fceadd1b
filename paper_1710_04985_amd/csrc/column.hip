// Column-wise solves on the level-ordered plan (Li, arXiv:1710.04985:
// Sec. 3.2 for the sweep, Sec. 4.1 LEVC, Sec. 4.2 SLFC).
//
// Position k holds acc[k] = b_i minus every update pushed so far (i the row
// solved at k).  Once all in-degree(k) updates have arrived, x_i = acc[k] *
// (1 / d_i); the column then adds -T(j,i) x_i to acc of each dependent position
// and, in the self-scheduled form, counts one arrival there.  The updates
// land in an order fixed by timing, so results match the row-wise solves to
// rounding, not bit for bit.
#include <hip/hip_runtime.h>

#include "column.hpp"
#include "residency.hpp"

namespace sptrsv {
namespace {

enum : int { kTimeout = kStatusTimeout };

template <typename T> __device__ __forceinline__ T load_agent_v(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int load_count(const int* p) {
  return __hip_atomic_load(const_cast<int*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait until *p == target; on timeout (or once another wavefront has
// timed out) raises TIMEOUT and returns, so the grid drains.
__device__ __attribute__((noinline)) void wait_count(const int* p, int target, int spin_limit,
                                                     int* status) {
  for (int s = 1; s <= spin_limit; ++s) {
    __builtin_amdgcn_s_sleep(1);
    if (load_count(p) == target) return;
    if ((s & 15) == 1 && (load_count(status) & kTimeout)) break;
  }
  __hip_atomic_fetch_or(status, kTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T> struct CArgs {
  const int* off_ptr;    // in-degree of position k = off_ptr[k+1] - off_ptr[k]
  const T* dinv;   // 1 / diagonal, by position
  const int* pos_row;
  const int* push_ptr;
  const int* push_dst;
  const T* push_val;
  const T* b;
  T* x;
  T* acc;
  int* cnt;
  int* status;
  int* arrive;
  int n;
  int spin_limit;
  int res_limit;
};

template <typename T>
__global__ void __launch_bounds__(256) k_push_gather(int64_t nnz, const int* __restrict__ src,
                                                     const T* __restrict__ off_val,
                                                     T* __restrict__ val) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < nnz;
       e += stride)
    val[e] = off_val[src[e]];
}

template <typename T> __global__ void __launch_bounds__(256) k_column_init(CArgs<T> a) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.arrive = 0;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < a.n;
       t += stride) {
    const int k = static_cast<int>(t);
    a.acc[k] = a.b[a.pos_row[k]];
    a.cnt[k] = 0;
  }
}

// Pushes x_k along the lane's entries e, e+G, ... of column k's list.  In the
// self-scheduled form each arrival count is raised only after the lane's
// value updates have returned (their results are consumed by an empty asm
// statement, which makes the compiler wait for them), so a consumer that
// sees the full count reads a complete accumulator.
template <typename T, bool kCount>
__device__ __forceinline__ void push_column(const CArgs<T>& a, int e, int e1, int G, T xk) {
  for (; e < e1; e += 4 * G) {
    int d[4];
    T u[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int eq = e + q * G;
      const bool on = eq < e1;
      d[q] = on ? a.push_dst[eq] : -1;
      u[q] = on ? -a.push_val[eq] * xk : T(0);
    }
    if (kCount) {
      T old[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        old[q] = d[q] >= 0 ? __hip_atomic_fetch_add(a.acc + d[q], u[q], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)
                           : T(0);
      int one = 1;
      __asm__ volatile("" : "+v"(one) : "v"(old[0]), "v"(old[1]), "v"(old[2]), "v"(old[3]));
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (d[q] >= 0)
          __hip_atomic_fetch_add(a.cnt + d[q], one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (d[q] >= 0)
          __hip_atomic_fetch_add(a.acc + d[q], u[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// One chunk: rows of G = 2^lg lanes, one column per row group.
template <typename T, bool kSelf>
__device__ __forceinline__ void column_chunk(const CArgs<T>& a, int st, int meta, int lane) {
  const int count = meta & 0xffff, lg = meta >> 16;
  const int G = 1 << lg;
  const int slot = lane >> lg, g = lane & (G - 1);
  if (slot >= count) return;
  const int k = st + slot;
  T v;
  if (kSelf) {
    const int indeg = a.off_ptr[k + 1] - a.off_ptr[k];
    if (indeg > 0 && load_count(a.cnt + k) != indeg)
      wait_count(a.cnt + k, indeg, a.spin_limit, a.status);
    v = load_agent_v(a.acc + k);
  } else {
    v = a.acc[k];
  }
  const T xk = v * a.dinv[k];
  if (g == 0) a.x[a.pos_row[k]] = xk;
  push_column<T, kSelf>(a, a.push_ptr[k] + g, a.push_ptr[k + 1], G, xk);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_column_level(CArgs<T> a, const int* __restrict__ cstart, const int* __restrict__ cmeta, int cb,
               int ce) {
  const int lane = threadIdx.x & 63;
  const int wave = static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int c = cb + wave;
  if (c >= ce) return;
  column_chunk<T, false>(a, cstart[c], cmeta[c], lane);
}

// Chunk c is handled by wavefront c mod W (lists in wptr/wlist, increasing),
// on an all-resident grid (checked at the start): the lowest unfinished
// chunk has all its columns' dependencies pushed and its wavefront working
// on it, so the solve progresses.
template <typename T>
__global__ void __launch_bounds__(256)
k_column_self(CArgs<T> a, const int* __restrict__ cstart, const int* __restrict__ cmeta,
              const int* __restrict__ wptr, const int* __restrict__ wlist) {
  const int lane = threadIdx.x & 63;
  if (!grid_resident(a.arrive, a.res_limit, a.status)) return;
  const int wave = static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lb = wptr[wave], le = wptr[wave + 1];
  for (int t = lb; t < le; ++t) {
    const int c = wlist[t];
    column_chunk<T, true>(a, cstart[c], cmeta[c], lane);
  }
}

template <typename T> CArgs<T> make_cargs(const ColumnArgs& s) {
  CArgs<T> a;
  a.off_ptr = s.plan->off_ptr;
  a.dinv = static_cast<const T*>(s.plan->dinv);
  a.pos_row = s.plan->pos_row;
  a.push_ptr = s.push->ptr;
  a.push_dst = s.push->dst;
  a.push_val = static_cast<const T*>(s.push->val);
  a.b = static_cast<const T*>(s.b);
  a.x = static_cast<T*>(s.x);
  a.acc = static_cast<T*>(s.acc);
  a.cnt = s.cnt;
  a.status = s.status;
  a.arrive = s.arrive;
  a.n = s.plan->n;
  a.spin_limit = s.spin_limit;
  a.res_limit = s.res_limit;
  return a;
}

inline int grid_for(int64_t work, int per_block, int cap) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  return static_cast<int>(b < cap ? b : cap);
}

}  // namespace

template <typename T>
hipError_t launch_push_gather(const DevPlan& p, const DevPush& q, hipStream_t s) {
  if (q.nnz == 0) return hipSuccess;
  k_push_gather<T><<<grid_for(q.nnz, 256, 65536), 256, 0, s>>>(
      q.nnz, q.src, static_cast<const T*>(p.off_val), static_cast<T*>(q.val));
  return hipGetLastError();
}

template <typename T> hipError_t launch_column_init(const ColumnArgs& sa, hipStream_t s) {
  if (sa.plan->n == 0) return hipSuccess;
  k_column_init<T><<<grid_for(sa.plan->n, 256, 8192), 256, 0, s>>>(make_cargs<T>(sa));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_column_level(const ColumnArgs& sa, int cb, int ce, hipStream_t s) {
  if (ce <= cb) return hipSuccess;
  const int wpb = sa.wg / 64;
  k_column_level<T><<<grid_for(ce - cb, wpb, 1 << 30), sa.wg, 0, s>>>(
      make_cargs<T>(sa), sa.chunks->start, sa.chunks->meta, cb, ce);
  return hipGetLastError();
}

template <typename T> hipError_t launch_column_self(const ColumnArgs& sa, hipStream_t s) {
  if (sa.chunks->count == 0) return hipSuccess;
  CArgs<T> ka = make_cargs<T>(sa);
  const int* cs = sa.chunks->start;
  const int* cm = sa.chunks->meta;
  const int* wp = sa.wave_ptr;
  const int* wl = sa.wave_list;
  void* args[] = {&ka, &cs, &cm, &wp, &wl};
  const void* fn = reinterpret_cast<const void*>(k_column_self<T>);
  if (sa.coop) return hipLaunchCooperativeKernel(fn, dim3(sa.grid), dim3(sa.wg), args, 0, s);
  return hipLaunchKernel(fn, dim3(sa.grid), dim3(sa.wg), args, 0, s);
}

template <typename T> int column_self_blocks_per_cu(int wg) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_column_self<T>, wg, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

#define SPTRSV_COLUMN_INSTANTIATE(T)                                                   \
  template hipError_t launch_push_gather<T>(const DevPlan&, const DevPush&, hipStream_t); \
  template hipError_t launch_column_init<T>(const ColumnArgs&, hipStream_t);           \
  template hipError_t launch_column_level<T>(const ColumnArgs&, int, int, hipStream_t); \
  template hipError_t launch_column_self<T>(const ColumnArgs&, hipStream_t);           \
  template int column_self_blocks_per_cu<T>(int);

SPTRSV_COLUMN_INSTANTIATE(double)
SPTRSV_COLUMN_INSTANTIATE(float)

}  // namespace sptrsv
