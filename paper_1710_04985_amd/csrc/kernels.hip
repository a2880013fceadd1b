// Solve kernels for gfx950 (CDNA4, 64-lane wavefronts).
//
// Work unit: a chunk = up to 64 consecutive level-ordered positions of ONE
// level; a wavefront takes a chunk and gives each row G = 2^lg lanes.  Lanes
// of a row stride over its off-diagonal entries (coalesced, the entries of a
// chunk are contiguous in the level-ordered copy), gather x at the entry's
// column, accumulate with FMA in a fixed order, and the group is summed with
// a butterfly of lane exchanges.  Every kernel that solves rows uses the same
// row_dot and group_sum, so at equal G the level-scheduled and the
// self-scheduled solves produce bit-identical x.
//
// Level-scheduled (Sec. 4.1, LEVR): one launch per level over its chunks;
// the launch boundary is the global synchronisation between levels.
//
// Self-scheduled (Sec. 4.2, SLFR): one persistent launch.  Wavefronts claim
// chunks from an atomic ticket in level order, the order of the paper's jlev
// mapping, so every row a claimed row waits for was claimed earlier by a
// running wavefront: the wait always ends (no co-residency assumption).
// Readiness of x_j is signalled either by x_j itself (x pre-filled with a
// signalling NaN that no arithmetic produces; x_j published by one
// agent-scope atomic store, polled with agent-scope atomic loads -- no cache
// maintenance), or by a per-row flag stamped with the solve's epoch and
// ordered by agent-scope release/acquire fences (the paper's dependency
// counter, without its per-solve reset).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace sptrsv {
namespace {

template <typename T> struct Bits;
template <> struct Bits<double> {
  using U = unsigned long long;
  // exponent all ones, quiet bit (51) clear, payload nonzero: a signalling NaN
  static constexpr U kSentinel = 0x7FF4A5A5A5A5A5A5ull;
};
template <> struct Bits<float> {
  using U = unsigned int;
  static constexpr U kSentinel = 0x7FA5A5A5u;   // quiet bit (22) clear
};

template <typename T> __device__ __forceinline__ T load_agent(const T* p) {
  using U = typename Bits<T>::U;
  const U u = __hip_atomic_load(reinterpret_cast<U*>(const_cast<T*>(p)), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(T, u);
}

template <typename T> __device__ __forceinline__ void store_agent(T* p, T v) {
  using U = typename Bits<T>::U;
  __hip_atomic_store(reinterpret_cast<U*>(p), __builtin_bit_cast(U, v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T> __device__ __forceinline__ bool is_sentinel(T v) {
  return __builtin_bit_cast(typename Bits<T>::U, v) == Bits<T>::kSentinel;
}

// quiets a signalling NaN, leaves every other value unchanged
__device__ __forceinline__ double canonical(double v) { return __builtin_canonicalize(v); }
__device__ __forceinline__ float canonical(float v) { return __builtin_canonicalizef(v); }

__device__ __forceinline__ int load_status(const int* s) {
  return __hip_atomic_load(const_cast<int*>(s), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void raise_status(int* s, int bit) {
  __hip_atomic_fetch_or(s, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait for x_j (value sync).  After spin_limit polls, or once another
// wavefront has timed out, the wait gives up: TIMEOUT is raised and a quiet
// NaN is used, so every dependent finishes and the grid drains.
template <typename T>
__device__ __attribute__((noinline)) T wait_value(const T* p, int spin_limit, int* status) {
  for (int s = 1; s <= spin_limit; ++s) {
    __builtin_amdgcn_s_sleep(1);
    const T v = load_agent(p);
    if (!is_sentinel(v)) return v;
    if ((s & 15) == 1 && (load_status(status) & kStatusTimeout)) break;
  }
  raise_status(status, kStatusTimeout);
  return __builtin_nan("");
}

// Bounded wait for flag[j] == epoch (flag sync); false on timeout.
__device__ __attribute__((noinline)) bool wait_flag(const unsigned* f, unsigned epoch,
                                                    int spin_limit, int* status) {
  for (int s = 1; s <= spin_limit; ++s) {
    __builtin_amdgcn_s_sleep(1);
    if (__hip_atomic_load(const_cast<unsigned*>(f), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
        epoch)
      return true;
    if ((s & 15) == 1 && (load_status(status) & kStatusTimeout)) break;
  }
  raise_status(status, kStatusTimeout);
  return false;
}

template <typename T> struct KArgs {
  const int* chunk_start;
  const int* chunk_meta;
  int nchunks;
  const int* off_ptr;
  const int* off_col;
  const T* off_val;
  const T* diag;
  const int* pos_row;
  const T* b;
  T* x;
  int ld;
  int nrhs;
  int* ticket;
  int* status;
  unsigned* epoch;
  unsigned* flags;
  int spin_limit;
};

// Sum over the lane's entries e0+gl, e0+gl+G, ... of val*x[col], in that
// order, four entries in flight at a time.  kPoll: x is read with agent-scope
// atomic loads and sentinel values are waited for.
template <typename T, bool kPoll>
__device__ __forceinline__ T row_dot(const int* __restrict__ off_col,
                                     const T* __restrict__ off_val, int e0, int e1, int gl,
                                     int G, const T* x, int spin_limit, int* status) {
  T sum = T(0);
  for (int e = e0 + gl; e < e1; e += 4 * G) {
    int j[4];
    T v[4], xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ee = e + u * G;
      j[u] = ee < e1 ? off_col[ee] : -1;
      v[u] = ee < e1 ? off_val[ee] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (j[u] >= 0) xv[u] = kPoll ? load_agent(x + j[u]) : x[j[u]];
      else xv[u] = T(0);
    }
    if constexpr (kPoll) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (j[u] >= 0 && is_sentinel(xv[u])) xv[u] = wait_value(x + j[u], spin_limit, status);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (j[u] >= 0) sum = __builtin_fma(v[u], xv[u], sum);
  }
  return sum;
}

template <typename T> __device__ __forceinline__ T group_sum(T v, int lg) {
  for (int o = 1; o < (1 << lg); o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Claims the next chunk for the calling wavefront (lane 0 does the atomic).
// Returns -1 when all chunks are taken; the very last claim of the grid
// resets the ticket for the next solve (all nchunks + nwaves claims happen,
// each wavefront ending with exactly one failing claim).
__device__ __forceinline__ int claim_chunk(int* ticket, int nchunks, int lane) {
  int c = 0;
  if (lane == 0) c = atomicAdd(ticket, 1);
  c = wave_uniform(c);
  if (c < nchunks) return c;
  const int nwaves = static_cast<int>(gridDim.x * (blockDim.x >> 6));
  if (lane == 0 && c == nchunks + nwaves - 1)
    __hip_atomic_store(ticket, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return -1;
}

// ---------------------------------------------------------------- level
template <typename T>
__global__ void __launch_bounds__(1024) k_level(KArgs<T> a, int chunk_begin, int chunk_end) {
  const int lane = threadIdx.x & 63;
  const int c = wave_uniform(chunk_begin + static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  if (c >= chunk_end) return;
  const int start = a.chunk_start[c];
  const int meta = a.chunk_meta[c];
  const int cnt = meta & 0xff, lg = meta >> 8;
  const int r = lane >> lg, gl = lane & ((1 << lg) - 1);
  const bool active = r < cnt;
  const int k = start + r;
  T sum = T(0);
  if (active)
    sum = row_dot<T, false>(a.off_col, a.off_val, a.off_ptr[k], a.off_ptr[k + 1], gl, 1 << lg,
                            a.x, 0, a.status);
  sum = group_sum(sum, lg);
  if (active && gl == 0) {
    const int i = a.pos_row[k];
    a.x[i] = canonical((a.b[i] - sum) / a.diag[k]);
  }
}

// ----------------------------------------------------- self, value sync
template <typename T>
__global__ void __launch_bounds__(1024) k_self_value(KArgs<T> a) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    const int c = claim_chunk(a.ticket, a.nchunks, lane);
    if (c < 0) return;
    const int start = a.chunk_start[c];
    const int meta = a.chunk_meta[c];
    const int cnt = meta & 0xff, lg = meta >> 8;
    const int r = lane >> lg, gl = lane & ((1 << lg) - 1);
    const bool active = r < cnt;
    const int k = start + r;
    T sum = T(0);
    if (active)
      sum = row_dot<T, true>(a.off_col, a.off_val, a.off_ptr[k], a.off_ptr[k + 1], gl, 1 << lg,
                             a.x, a.spin_limit, a.status);
    sum = group_sum(sum, lg);
    if (active && gl == 0) {
      const int i = a.pos_row[k];
      store_agent(a.x + i, canonical((a.b[i] - sum) / a.diag[k]));
    }
  }
}

// ------------------------------------------------------ self, flag sync
template <typename T>
__global__ void __launch_bounds__(1024) k_self_flag(KArgs<T> a) {
  const int lane = threadIdx.x & 63;
  const unsigned epoch = *a.epoch;
  for (;;) {
    int c = 0;
    if (lane == 0) c = atomicAdd(a.ticket, 1);
    c = wave_uniform(c);
    if (c >= a.nchunks) {
      const int nwaves = static_cast<int>(gridDim.x * (blockDim.x >> 6));
      if (lane == 0 && c == a.nchunks + nwaves - 1) {
        // last claim of the grid: next solve gets a fresh epoch and ticket
        const unsigned nxt = epoch + 1u == 0u ? 1u : epoch + 1u;
        __hip_atomic_store(a.epoch, nxt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.ticket, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      return;
    }
    const int start = a.chunk_start[c];
    const int meta = a.chunk_meta[c];
    const int cnt = meta & 0xff, lg = meta >> 8;
    const int G = 1 << lg;
    const int r = lane >> lg, gl = lane & (G - 1);
    const bool active = r < cnt;
    const int k = start + r;
    int e0 = 0, e1 = 0;
    if (active) {
      e0 = a.off_ptr[k];
      e1 = a.off_ptr[k + 1];
      for (int e = e0 + gl; e < e1; e += G) {
        const unsigned* f = a.flags + a.off_col[e];
        if (__hip_atomic_load(const_cast<unsigned*>(f), __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT) != epoch)
          wait_flag(f, epoch, a.spin_limit, a.status);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    T sum = T(0);
    if (active) sum = row_dot<T, false>(a.off_col, a.off_val, e0, e1, gl, G, a.x, 0, a.status);
    sum = group_sum(sum, lg);
    int i = -1;
    if (active && gl == 0) {
      i = a.pos_row[k];
      a.x[i] = canonical((a.b[i] - sum) / a.diag[k]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (i >= 0)
      __hip_atomic_store(a.flags + i, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// -------------------------------------------------- multi-RHS (columns)
// Lanes of a row take right-hand sides (KL = 2^lg lanes, RHS q = lane % KL
// + multiples of KL); each lane runs the whole row for its column, so the
// row's indices and values are loaded once per wavefront for all columns.
template <typename T, bool kPoll>
__device__ __forceinline__ void multi_rows(const KArgs<T>& a, int c, int lane) {
  const int start = a.chunk_start[c];
  const int meta = a.chunk_meta[c];
  const int cnt = meta & 0xff, lg = meta >> 8;
  const int r = lane >> lg, q0 = lane & ((1 << lg) - 1);
  if (r >= cnt) return;
  const int k = start + r;
  const int i = a.pos_row[k];
  const int e0 = a.off_ptr[k], e1 = a.off_ptr[k + 1];
  const T d = a.diag[k];
  for (int q = q0; q < a.nrhs; q += (1 << lg)) {
    const size_t off = static_cast<size_t>(q) * a.ld;
    const T sum = row_dot<T, kPoll>(a.off_col, a.off_val, e0, e1, 0, 1, a.x + off, a.spin_limit,
                                    a.status);
    const T xi = canonical((a.b[off + i] - sum) / d);
    if (kPoll) store_agent(a.x + off + i, xi);
    else a.x[off + i] = xi;
  }
}

template <typename T>
__global__ void __launch_bounds__(1024) k_level_multi(KArgs<T> a, int chunk_begin, int chunk_end) {
  const int lane = threadIdx.x & 63;
  const int c = wave_uniform(chunk_begin + static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  if (c >= chunk_end) return;
  multi_rows<T, false>(a, c, lane);
}

template <typename T>
__global__ void __launch_bounds__(1024) k_self_multi_value(KArgs<T> a) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    const int c = claim_chunk(a.ticket, a.nchunks, lane);
    if (c < 0) return;
    multi_rows<T, true>(a, c, lane);
  }
}

// ------------------------------------------------------------ utilities
template <typename T>
__global__ void __launch_bounds__(256) k_gather(int64_t noff, int n, const int* __restrict__ off_src,
                                                const int* __restrict__ diag_src,
                                                const T* __restrict__ vals, T* __restrict__ off_val,
                                                T* __restrict__ diag, int* status) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t total = noff > n ? noff : n;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += stride) {
    if (t < noff) off_val[t] = vals[off_src[t]];
    if (t < n) {
      const int s = diag_src[t];
      const T d = s >= 0 ? vals[s] : T(1);
      diag[t] = d;
      if (d == T(0)) raise_status(status, kStatusZeroPivot);
    }
  }
}

// x := sentinel over n rows of each column (column stride ld); when save is
// given, the previous contents are copied there first (in-place solves).
template <typename T>
__global__ void __launch_bounds__(256) k_fill_sentinel(T* x, T* save, int n, int ld) {
  using U = typename Bits<T>::U;
  const size_t off = static_cast<size_t>(blockIdx.y) * ld;
  U* xc = reinterpret_cast<U*>(x + off);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (save) save[off + i] = x[off + i];
    xc[i] = Bits<T>::kSentinel;
  }
}

// grad_vals[e] = -grad_b[i] * x[col[e]] over the caller's CSR, 4 lanes a row
template <typename T>
__global__ void __launch_bounds__(256) k_grad_vals(int n, const int* __restrict__ row_ptr,
                                                   const int* __restrict__ col, int unit_diag,
                                                   const T* __restrict__ grad_b,
                                                   const T* __restrict__ x,
                                                   T* __restrict__ grad_vals) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t >> 2, gl = t & 3;
  if (i >= n) return;
  const T g = -grad_b[i];
  for (int e = row_ptr[i] + gl; e < row_ptr[i + 1]; e += 4) {
    const int j = col[e];
    grad_vals[e] = (unit_diag && j == i) ? T(0) : g * x[j];
  }
}

__global__ void __launch_bounds__(256) k_init_scratch(int* ticket, int* status, unsigned* epoch,
                                                      unsigned* flags, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    *ticket = 0;
    *status = 0;
    *epoch = 1u;
  }
  for (int i = t; i < n; i += gridDim.x * blockDim.x) flags[i] = 0u;
}

template <typename T> KArgs<T> make_args(const SolveArgs& s) {
  KArgs<T> a;
  a.chunk_start = s.chunks->start;
  a.chunk_meta = s.chunks->meta;
  a.nchunks = s.chunks->count;
  a.off_ptr = s.plan->off_ptr;
  a.off_col = s.plan->off_col;
  a.off_val = static_cast<const T*>(s.plan->off_val);
  a.diag = static_cast<const T*>(s.plan->diag);
  a.pos_row = s.plan->pos_row;
  a.b = static_cast<const T*>(s.b);
  a.x = static_cast<T*>(s.x);
  a.ld = s.ld;
  a.nrhs = s.nrhs;
  a.ticket = s.scratch.ticket;
  a.status = s.scratch.status;
  a.epoch = s.scratch.epoch;
  a.flags = s.scratch.flags;
  a.spin_limit = s.spin_limit;
  return a;
}

inline int blocks_for(int64_t work, int per_block, int cap) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  return static_cast<int>(b < cap ? b : cap);
}

}  // namespace

template <typename T>
hipError_t launch_gather(const DevPlan& p, const T* vals, int* status, hipStream_t s) {
  const int64_t total = p.noff > p.n ? p.noff : p.n;
  if (total == 0) return hipSuccess;
  k_gather<T><<<blocks_for(total, 256, 65536), 256, 0, s>>>(
      p.noff, p.n, p.off_src, p.diag_src, vals, static_cast<T*>(p.off_val),
      static_cast<T*>(p.diag), status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_sentinel(T* x, T* save, int n, int nrhs, int ld, hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  dim3 grid(blocks_for(n, 256, 8192), nrhs);
  k_fill_sentinel<T><<<grid, 256, 0, s>>>(x, save, n, ld);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_level(const SolveArgs& sa, int cb, int ce, hipStream_t s) {
  if (ce <= cb) return hipSuccess;
  const int wpb = sa.wg / 64;
  k_level<T><<<blocks_for(ce - cb, wpb, 1 << 30), sa.wg, 0, s>>>(make_args<T>(sa), cb, ce);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_level_multi(const SolveArgs& sa, int cb, int ce, hipStream_t s) {
  if (ce <= cb) return hipSuccess;
  const int wpb = sa.wg / 64;
  k_level_multi<T><<<blocks_for(ce - cb, wpb, 1 << 30), sa.wg, 0, s>>>(make_args<T>(sa), cb, ce);
  return hipGetLastError();
}

template <typename T> hipError_t launch_self_value(const SolveArgs& sa, hipStream_t s) {
  if (sa.chunks->count == 0) return hipSuccess;
  k_self_value<T><<<sa.grid, sa.wg, 0, s>>>(make_args<T>(sa));
  return hipGetLastError();
}

template <typename T> hipError_t launch_self_flag(const SolveArgs& sa, hipStream_t s) {
  if (sa.chunks->count == 0) return hipSuccess;
  k_self_flag<T><<<sa.grid, sa.wg, 0, s>>>(make_args<T>(sa));
  return hipGetLastError();
}

template <typename T> hipError_t launch_self_multi_value(const SolveArgs& sa, hipStream_t s) {
  if (sa.chunks->count == 0) return hipSuccess;
  k_self_multi_value<T><<<sa.grid, sa.wg, 0, s>>>(make_args<T>(sa));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_grad_vals(int n, const int* row_ptr, const int* col, int unit_diag,
                            const T* grad_b, const T* x, T* grad_vals, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_grad_vals<T><<<blocks_for(static_cast<int64_t>(n) * 4, 256, 1 << 30), 256, 0, s>>>(
      n, row_ptr, col, unit_diag, grad_b, x, grad_vals);
  return hipGetLastError();
}

hipError_t launch_init_scratch(DevScratch sc, int n, hipStream_t s) {
  k_init_scratch<<<blocks_for(n > 0 ? n : 1, 256, 4096), 256, 0, s>>>(sc.ticket, sc.status,
                                                                      sc.epoch, sc.flags, n);
  return hipGetLastError();
}

template <typename T> int self_value_blocks_per_cu(int wg) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_self_value<T>, wg, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}
template <typename T> int self_flag_blocks_per_cu(int wg) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_self_flag<T>, wg, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}
template <typename T> int self_multi_blocks_per_cu(int wg) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_self_multi_value<T>, wg, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

#define SPTRSV_INSTANTIATE(T)                                                                   \
  template hipError_t launch_gather<T>(const DevPlan&, const T*, int*, hipStream_t);            \
  template hipError_t launch_fill_sentinel<T>(T*, T*, int, int, int, hipStream_t);              \
  template hipError_t launch_level<T>(const SolveArgs&, int, int, hipStream_t);                 \
  template hipError_t launch_level_multi<T>(const SolveArgs&, int, int, hipStream_t);           \
  template hipError_t launch_self_value<T>(const SolveArgs&, hipStream_t);                      \
  template hipError_t launch_self_flag<T>(const SolveArgs&, hipStream_t);                       \
  template hipError_t launch_self_multi_value<T>(const SolveArgs&, hipStream_t);                \
  template hipError_t launch_grad_vals<T>(int, const int*, const int*, int, const T*, const T*, \
                                          T*, hipStream_t);                                     \
  template int self_value_blocks_per_cu<T>(int);                                                \
  template int self_flag_blocks_per_cu<T>(int);                                                 \
  template int self_multi_blocks_per_cu<T>(int);

SPTRSV_INSTANTIATE(double)
SPTRSV_INSTANTIATE(float)

}  // namespace sptrsv
