// Solve kernels for gfx950 (CDNA4, 64-lane wavefronts).
//
// Work unit: a chunk = consecutive level-ordered positions of ONE level (see
// the chunk encoding in analysis.hpp); a wavefront takes a chunk.  With one
// right-hand side a row gets G = 2^lg lanes that stride its off-diagonal
// entries (coalesced: the entries of a chunk are contiguous in the
// level-ordered copy), gather x, accumulate with FMA in a fixed order, and a
// butterfly of lane exchanges sums the group; with G = 1 a lane may own
// several rows.  With several right-hand sides the lanes of a row take
// columns instead and each walks the whole row.  Every kernel uses the same
// per-row order, so at equal chunking the schedules agree bit for bit.
// A row's value is (b_i - sum) times the reciprocal of its diagonal, which
// the value gather computes once (the form of the paper's SLFR listing,
// Sec. 4.2): it takes the division's dependent instruction chain off the
// critical path of every row; the result is within 1.5 units in the last
// place of the divided one.
//
// The solution is kept in position order (xp, see SolveArgs): dependencies of
// neighbouring rows of a level are neighbouring positions of earlier levels,
// so the x gathers coalesce.  Each row is also written to the caller's x.
//
// Level-scheduled (Sec. 4.1, LEVR): one launch per level over its chunks;
// the launch boundary is the global synchronisation between levels.
//
// Self-scheduled (Sec. 4.2, SLFR): one persistent launch; wavefronts take
// chunks in level order, the order of the paper's jlev mapping, and wait for
// the individual rows they depend on.  Readiness of a row is signalled by
// its value itself: xp starts filled with a signalling NaN that no
// arithmetic produces, each value is published by one agent-scope atomic
// store and polled with agent-scope atomic loads, so no cache maintenance is
// needed.  The paper's dependency counters are also available as per-row
// flags stamped with the solve's epoch, ordered by agent-scope
// release/acquire fences (flag sync).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "analysis.hpp"
#include "kernels.hpp"
#include "residency.hpp"

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

// fused multiply-add in the value type (FP64 or FP32: one rounding, no
// widening)
__device__ __forceinline__ double fma_t(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
__device__ __forceinline__ float fma_t(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
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

// Joint bounded wait for the dependencies j[0..N) whose values in xv are
// still the sentinel.  Two polling modes (a schedule option):
//  overlap: every round polls all N values (unconditionally, so the number of
//    loads in flight is fixed) and two rounds overlap: round r+1 is issued
//    before round r's results are examined, so a value published while a poll
//    is in flight is seen about one interval later instead of one full round
//    trip later.  Best when most of a lane's dependencies are pending
//    (mesh-like triangles).
//  single: one round at a time, polling only the values still pending.  Less
//    polling traffic; best when most dependencies are already available
//    (irregular triangles whose dependencies span many levels).
// Either way the wait ends soon after the last pending value is published.
// After spin_limit rounds, or once another wavefront has timed out, TIMEOUT
// is raised and the pending values become quiet NaNs, so the grid drains.
template <typename T, int N>
__device__ __forceinline__ void wait_values(const T* xr, int xs, const int (&j)[N], T (&xv)[N],
                                            int spin_limit, int* status, bool overlap) {
  unsigned pend = 0;
#pragma unroll
  for (int q = 0; q < N; ++q)
    if (j[q] >= 0 && is_sentinel(xv[q])) pend |= 1u << q;
  if (!pend) return;
  const T* p[N];
#pragma unroll
  for (int q = 0; q < N; ++q) p[q] = xr + static_cast<int64_t>(j[q] >= 0 ? j[q] : 0) * xs;
  auto take = [&](const T (&v)[N]) {
#pragma unroll
    for (int q = 0; q < N; ++q)
      if (((pend >> q) & 1u) && !is_sentinel(v[q])) {
        xv[q] = v[q];
        pend &= ~(1u << q);
      }
  };
  if (overlap) {
    // two register sets polled in turn, so no copy forces a wait on the newer set
    T pa[N], pb[N];
#pragma unroll
    for (int q = 0; q < N; ++q) pa[q] = load_agent(p[q]);
    for (int s = 1; s <= spin_limit; s += 2) {
      __builtin_amdgcn_s_sleep(1);
#pragma unroll
      for (int q = 0; q < N; ++q) pb[q] = load_agent(p[q]);
      take(pa);
      if (!pend) return;
      __builtin_amdgcn_s_sleep(1);
#pragma unroll
      for (int q = 0; q < N; ++q) pa[q] = load_agent(p[q]);
      take(pb);
      if (!pend) return;
      // the status word only every 32 passes, and not in the first: waiting
      // for its load also waits for every poll in flight
      if ((s & 63) == 63 && (load_status(status) & kStatusTimeout)) break;
    }
  } else {
    for (int s = 1; s <= spin_limit; ++s) {
      __builtin_amdgcn_s_sleep(1);
      T nv[N];
#pragma unroll
      for (int q = 0; q < N; ++q) nv[q] = (pend >> q) & 1u ? load_agent(p[q]) : xv[q];
      take(nv);
      if (!pend) return;
      if ((s & 15) == 1 && (load_status(status) & kStatusTimeout)) break;
    }
  }
  raise_status(status, kStatusTimeout);
#pragma unroll
  for (int q = 0; q < N; ++q)
    if ((pend >> q) & 1u) xv[q] = __builtin_nan("");
}

template <typename T> struct KArgs {
  const int* chunk_start;
  const int* chunk_meta;
  int nchunks;
  int n;
  int64_t noff;
  const int* off_ptr;
  const int* off_col;
  const int* off_pos;
  const T* off_val;
  const T* dinv;          // 1 / diagonal, by position
  const int* pos_row;
  const T* b;
  T* x;
  T* xp;
  const T* bp;            // several right-hand sides: bp[k * nrhs + q], position order
  int ld;
  int nrhs;
  int* ticket;
  int* status;
  unsigned* epoch;
  unsigned* flags;
  int* arrive;
  int res_limit;
  int spin_limit;
  int poll;          // 1: overlapped polling of all slots, 0: single rounds of pending ones
  const int* chunk_col;   // column-batched tables: right-hand side of each chunk
  int64_t xp_col;         // elements between the columns of xp (column-batched)
};

// Continues `sum` over the lane's entries e, e+G, e+2G, ... < e1 of one row,
// four entries at a time, reading x at xr[idx[entry] * xs].  The indices and
// values of the next four entries are loaded while the x gathers of the
// current four are in flight, so a long row costs about one load round trip
// per four entries of the lane.  Accumulation is in entry order.
// kPoll: atomic agent-scope loads, sentinel values are waited for.  B
// entries per batch (more gathers in flight per lane for long rows; the
// level-scheduled kernels take 16, the polling ones 4, where more registers
// cost more than they save).  B does not change the order of the sum.
template <typename T, bool kPoll, int B = 4>
__device__ __forceinline__ T row_dot(const int* __restrict__ idx, const T* __restrict__ off_val,
                                     int e, int e1, int G, const T* xr, int xs, int spin_limit,
                                     int* status, bool overlap, T sum) {
  if (e >= e1) return sum;
  int j[B];
  T v[B];
#pragma unroll
  for (int u = 0; u < B; ++u) {
    const int ee = e + u * G;
    j[u] = ee < e1 ? idx[ee] : -1;
    v[u] = ee < e1 ? off_val[ee] : T(0);
  }
  for (;;) {
    T xv[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const T* p = xr + static_cast<int64_t>(j[u]) * xs;
      if (j[u] >= 0) xv[u] = kPoll ? load_agent(p) : *p;
      else xv[u] = T(0);
    }
    // next batch, only if the lane has one (its loads overlap the gathers above)
    const bool more = e + B * G < e1;
    int jn[B];
    T vn[B];
    if (more) {
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int ee = e + (B + u) * G;
        jn[u] = ee < e1 ? idx[ee] : -1;
        vn[u] = ee < e1 ? off_val[ee] : T(0);
      }
    }
    if constexpr (kPoll) wait_values<T, B>(xr, xs, j, xv, spin_limit, status, overlap);
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (j[u] >= 0) sum = fma_t(v[u], xv[u], sum);
    if (!more) break;
#pragma unroll
    for (int u = 0; u < B; ++u) {
      j[u] = jn[u];
      v[u] = vn[u];
    }
    e += B * G;
  }
  return sum;
}

template <typename T> __device__ __forceinline__ T group_sum(T v, int lg) {
  for (int o = 1; o < (1 << lg); o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T, bool kPoll> __device__ __forceinline__ void publish(T* p, T v) {
  if constexpr (kPoll) store_agent(p, v);
  else *p = v;
}

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Solves the rows of one chunk, one right-hand side.
//  G = 1: lane l owns rows start+l, start+l+64, ... (up to kMaxRowsPerLane);
//         bounds, first four entries, x gathers, b and diagonal of all its
//         rows are issued before any wait, then each row is finished.
//  G > 1: rows of G lanes; lanes stride the row, the group sums by butterfly.
template <typename T, bool kPoll, int RB = 4>
__device__ __forceinline__ void solve_chunk(const KArgs<T>& a, int start, int meta, int lane) {
  const int cnt = meta & 0xffff, lg = meta >> 16;
  if (lg == 0) {
    constexpr int R = kMaxRowsPerLane;
    constexpr int E = 4;
    int k[R], e0[R], e1[R], i[R];
    T bi[R], di[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int rr = lane + 64 * u;
      k[u] = rr < cnt ? start + rr : -1;
      e0[u] = 0;
      e1[u] = 0;
      i[u] = 0;
      bi[u] = T(0);
      di[u] = T(1);
      if (k[u] >= 0) {
        e0[u] = a.off_ptr[k[u]];
        e1[u] = a.off_ptr[k[u] + 1];
        i[u] = a.pos_row[k[u]];
        di[u] = a.dinv[k[u]];
      }
    }
    int j[R][E];
    T v[R][E], xv[R][E];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (k[u] >= 0) bi[u] = a.b[i[u]];
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int ee = e0[u] + q;
        j[u][q] = ee < e1[u] ? a.off_pos[ee] : -1;
        v[u][q] = ee < e1[u] ? a.off_val[ee] : T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
      for (int q = 0; q < E; ++q)
        xv[u][q] = j[u][q] >= 0 ? (kPoll ? load_agent(a.xp + j[u][q]) : a.xp[j[u][q]]) : T(0);
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (k[u] < 0) continue;
      T sum = T(0);
      if (kPoll) wait_values<T, E>(a.xp, 1, j[u], xv[u], a.spin_limit, a.status, a.poll != 0);
#pragma unroll
      for (int q = 0; q < E; ++q) {
        if (j[u][q] < 0) continue;
        sum = fma_t(v[u][q], xv[u][q], sum);
      }
      if (e1[u] > e0[u] + E)
        sum = row_dot<T, kPoll, RB>(a.off_pos, a.off_val, e0[u] + E, e1[u], 1, a.xp, 1,
                                    a.spin_limit, a.status, a.poll != 0, sum);
      const T xi = canonical((bi[u] - sum) * di[u]);
      publish<T, kPoll>(a.xp + k[u], xi);
      a.x[i[u]] = xi;
    }
    return;
  }
  const int r = lane >> lg, gl = lane & ((1 << lg) - 1);
  const bool active = r < cnt;
  const int k = start + r;
  T sum = T(0);
  if (active)
    sum = row_dot<T, kPoll, RB>(a.off_pos, a.off_val, a.off_ptr[k] + gl, a.off_ptr[k + 1],
                                1 << lg, a.xp, 1, a.spin_limit, a.status, a.poll != 0, T(0));
  sum = group_sum(sum, lg);
  if (active && gl == 0) {
    const int i = a.pos_row[k];
    const T xi = canonical((a.b[i] - sum) * a.dinv[k]);
    publish<T, kPoll>(a.xp + k, xi);
    a.x[i] = xi;
  }
}

// Several right-hand sides, in position order (bp in, xp out; see
// launch_multi_in / launch_multi_out): the 2^lg lanes of a row take columns
// q0 = lane % 2^lg (+ multiples of 2^lg); each lane walks all entries of its
// row in order for its column, so every column is solved as the
// one-lane-per-row single solve.  The row's indices and values are fetched
// once for all columns.
template <typename T, bool kPoll>
__device__ __forceinline__ void solve_chunk_multi(const KArgs<T>& a, int start, int meta,
                                                  int lane) {
  const int cnt = meta & 0xffff, lg = meta >> 16;
  const int r = lane >> lg, q0 = lane & ((1 << lg) - 1);
  if (r >= cnt) return;
  const int k = start + r;
  const int e0 = a.off_ptr[k], e1 = a.off_ptr[k + 1];
  const T d = a.dinv[k];
  for (int q = q0; q < a.nrhs; q += (1 << lg)) {
    const int64_t kq = static_cast<int64_t>(k) * a.nrhs + q;
    const T sum = row_dot<T, kPoll>(a.off_pos, a.off_val, e0, e1, 1, a.xp + q, a.nrhs,
                                    a.spin_limit, a.status, a.poll != 0, T(0));
    const T xi = canonical((a.bp[kq] - sum) * d);
    publish<T, kPoll>(a.xp + kq, xi);
  }
}

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
template <typename T, bool kMulti>
__global__ void __launch_bounds__(256) k_level(KArgs<T> a, int chunk_begin, int chunk_end) {
  const int lane = threadIdx.x & 63;
  const int c = wave_uniform(chunk_begin + static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  if (c >= chunk_end) return;
  if constexpr (kMulti) solve_chunk_multi<T, false>(a, a.chunk_start[c], a.chunk_meta[c], lane);
  else solve_chunk<T, false, 16>(a, a.chunk_start[c], a.chunk_meta[c], lane);
}

// Level-scheduled, one lane per row, one right-hand side: the rows of a
// level are the positions [k0, k1), one per thread, so no chunk descriptor
// sits in front of the row's loads.  Same per-row arithmetic as solve_chunk
// with one lane per row (first four entries, then the rest of the row in
// order, FMA from zero).
template <typename T>
__global__ void __launch_bounds__(256) k_level_flat(KArgs<T> a, int k0, int k1) {
  const int k = k0 + static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (k >= k1) return;
  const int e0 = a.off_ptr[k], e1 = a.off_ptr[k + 1];
  const int i = a.pos_row[k];
  const T d = a.dinv[k];
  int j[4];
  T v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ee = e0 + q;
    j[q] = ee < e1 ? a.off_pos[ee] : -1;
    v[q] = ee < e1 ? a.off_val[ee] : T(0);
  }
  const T bi = a.b[i];
  T xv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) xv[q] = j[q] >= 0 ? a.xp[j[q]] : T(0);
  T sum = T(0);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (j[q] >= 0) sum = fma_t(v[q], xv[q], sum);
  if (e1 > e0 + 4)
    sum = row_dot<T, false, 16>(a.off_pos, a.off_val, e0 + 4, e1, 1, a.xp, 1, a.spin_limit,
                                a.status, false, sum);
  const T xi = canonical((bi - sum) * d);
  a.xp[k] = xi;
  a.x[i] = xi;
}

// ------------------------------------------------ self, value sync, ticket
template <typename T, bool kMulti>
__global__ void __launch_bounds__(256) k_self_value(KArgs<T> a) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    const int c = claim_chunk(a.ticket, a.nchunks, lane);
    if (c < 0) return;
    if constexpr (kMulti) solve_chunk_multi<T, true>(a, a.chunk_start[c], a.chunk_meta[c], lane);
    else solve_chunk<T, true>(a, a.chunk_start[c], a.chunk_meta[c], lane);
  }
}

// ------------------------------------- self, value sync, static pipeline
// Wavefront w takes the chunks of its own list in increasing order (lists are
// fixed before the launch: round-robin, or by XCD region).  All wavefronts of
// the grid are resident (it is sized well below the occupancy figure, and
// each wavefront checks at its start that the whole grid has signed in), so
// the wavefront holding the lowest unfinished chunk has finished its earlier
// chunks and is working on it, and that chunk's dependencies are done.  No
// claim atomics.
// Each chunk moves through four stages, one chunk apart, so the dependent
// index loads of later chunks are in flight while this one waits on x:
//   A descriptor -> B row bounds, row, diagonal -> C first entries, b
//   -> D gather x (poll), accumulate, publish.
// Each stage only stores raw loaded values; any arithmetic on them happens
// one iteration later, so no wait for a load is needed before the next
// stage's loads (and the x gathers) have been issued.  Loads whose result is
// discarded use clamped in-range indices instead of branches.  One
// right-hand side (k_self_multi takes several).
template <typename T> struct StageB {   // descriptor, raw
  int c, start, meta, q;
};
template <typename T> struct StageC {   // row bounds, raw
  int c, meta, k, p0, p1, i;
  T d;
  int q;
};
template <typename T> struct StageD {   // first entries of the lane, raw
  int c, lg, k, e, e1, i;
  T d, bi;
  int j[4];
  T v[4];
  int q;
};

template <typename T, int kStride, bool kCols>
__global__ void __launch_bounds__(256)
k_self_static(KArgs<T> a, const int* __restrict__ cstart, const int* __restrict__ cmeta,
              const int* __restrict__ wptr, const int* __restrict__ wlist) {
  const int lane = threadIdx.x & 63;
  if (!grid_resident(a.arrive, a.res_limit, a.status)) return;
  const int w = wave_uniform(static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  // this wavefront's chunks: wlist[wptr[w] .. wptr[w+1]), increasing
  const int tb = wptr[w], te = wptr[w + 1];
  const int llast = a.nchunks - 1;    // clamp for the list load past the end
  const int nlast = a.n - 1;          // clamp for loads whose result is discarded
  const int64_t olast = a.noff > 0 ? a.noff - 1 : 0;
  const int xs = kStride;             // elements between xp values
  StageB<T> sb{-1, 0, 0, 0};
  StageC<T> sc{-1, 0, -1, 0, 0, 0, T(1), 0};
  StageD<T> sd;
  sd.c = -1;
  sd.lg = 0;
  sd.k = -1;
  sd.q = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) sd.j[q] = -1;
  int t = tb;                         // list index of the chunk entering stage A
  int cur = wlist[tb < te ? tb : llast];   // that chunk (loaded one iteration ahead)
  for (;;) {
    // ---- A: descriptor of a new chunk (uniform index, read-only tables)
    StageB<T> nb{-1, 0, 0, 0};
    {
      const bool live = t < te;
      const int cn = wave_uniform(cur);
      nb.start = cstart[cn];
      nb.meta = cmeta[cn];
      if constexpr (kCols) nb.q = a.chunk_col[cn];
      if (live) {
        nb.c = cn;
        ++t;
      }
      cur = wlist[t < te ? t : llast];
    }
    // ---- D (issue): gather x for the chunk whose entries arrived last time
    const T* xq = kCols ? a.xp + static_cast<int64_t>(sd.q) * a.xp_col : a.xp;
    T xv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      xv[q] = load_agent(xq + static_cast<int64_t>(sd.j[q] >= 0 ? sd.j[q] : 0) * xs);
    // ---- B: row bounds, row and diagonal of the chunk described last time
    StageC<T> nc{sb.c, sb.meta, -1, 0, 0, 0, T(1), sb.q};
    {
      const int lg = sb.meta >> 16, cnt = sb.meta & 0xffff;
      const int r = lane >> lg;
      const bool live = sb.c >= 0 && r < cnt;
      const int kk = live ? sb.start + r : nlast;
      nc.k = live ? kk : -1;
      nc.p0 = a.off_ptr[kk];
      nc.p1 = a.off_ptr[kk + 1];
      nc.i = a.pos_row[kk];
      nc.d = a.dinv[kk];
    }
    // ---- C: the lane's first four entries and b of the chunk bounded last time
    StageD<T> nd;
    nd.c = sc.c;
    nd.lg = sc.meta >> 16;
    nd.k = sc.k;
    nd.i = sc.i;
    nd.d = sc.d;
    nd.q = sc.q;
    {
      const int G = 1 << nd.lg;                       // entry stride of the lane
      const int gl = lane & (G - 1);
      nd.e = sc.p0 + gl;
      nd.e1 = sc.p1;
      const bool live = sc.c >= 0 && sc.k >= 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ee = nd.e + q * G;
        const bool ok = live && ee < nd.e1;
        const int64_t ec = ok ? ee : olast;
        const int jj = a.off_pos[ec];
        const T vv = a.off_val[ec];
        nd.j[q] = ok ? jj : -1;
        nd.v[q] = ok ? vv : T(0);
      }
      const T* bq = kCols ? a.b + static_cast<int64_t>(sc.q) * a.ld : a.b;
      const T bb = bq[sc.i];
      nd.bi = (live && gl == 0) ? bb : T(0);
    }
    // ---- D (finish): wait, accumulate, rest of the row, group sum, publish
    if (sd.c >= 0) {
      const int G = 1 << sd.lg;
      T sum = T(0);
      if (sd.k >= 0) {
        wait_values<T, 4>(xq, xs, sd.j, xv, a.spin_limit, a.status, a.poll != 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (sd.j[q] < 0) continue;
          sum = fma_t(sd.v[q], xv[q], sum);
        }
        if (sd.e + 4 * G < sd.e1)
          sum = row_dot<T, true>(a.off_pos, a.off_val, sd.e + 4 * G, sd.e1, G, xq, xs,
                                 a.spin_limit, a.status, a.poll != 0, sum);
      }
      sum = group_sum(sum, sd.lg);
      if (sd.k >= 0 && (lane & (G - 1)) == 0) {
        const T xi = canonical((sd.bi - sum) * sd.d);
        const int64_t qo = kCols ? static_cast<int64_t>(sd.q) : 0;
        store_agent(a.xp + qo * a.xp_col + static_cast<int64_t>(sd.k) * xs, xi);
        a.x[qo * a.ld + sd.i] = xi;
      }
    } else if (sc.c < 0 && sb.c < 0 && nb.c < 0) {
      return;                         // pipeline drained
    }
    sd = nd;
    sc = nc;
    sb = nb;
  }
}

// ------------------------- self, value sync, static pipeline, several RHS
// The static schedule of k_self_static for several right-hand sides, in
// position order: the right-hand sides come permuted into bp[k * nrhs + q]
// and the solution stays in xp[k * nrhs + q] (launch_multi_in and
// launch_multi_out move them from and to the caller's column-major B and X
// with coalesced passes), so every access of a chunk is contiguous.  The 2^lg
// lanes of a row take columns q = lane % 2^lg (2^lg >= nrhs, at most 64), so
// a chunk has 64 >> lg lane groups, each owning R rows of it (rows g,
// g + (64 >> lg), ...); a lane issues the x gathers of all R rows before it
// waits on any.  Column q of a row walks all entries in stored order with
// FMA, exactly as the one-lane single-RHS solve, so every column equals that
// solve bit for bit.  Columns beyond the first 2^lg are finished by the same
// lanes, unpipelined.  Same four stages as k_self_static (descriptor -> row
// bounds -> first entries and b -> gather, wait, publish), one chunk apart.
template <typename T, int R> struct MStageC {   // row bounds of R rows, raw
  int c, meta;
  int k[R], p0[R], p1[R];
  T d[R];
};
template <typename T, int R> struct MStageD {   // first entries of R rows, raw
  int c, lg;
  int k[R], e[R], e1[R];
  T d[R], bi[R];
  int j[R][4];
  T v[R][4];
};

template <typename T, int R>
__global__ void __launch_bounds__(256)
k_self_multi(KArgs<T> a, const int* __restrict__ cstart, const int* __restrict__ cmeta,
             const int* __restrict__ wptr, const int* __restrict__ wlist) {
  const int lane = threadIdx.x & 63;
  if (!grid_resident(a.arrive, a.res_limit, a.status)) return;
  const int w = wave_uniform(static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const int tb = wptr[w], te = wptr[w + 1];
  const int llast = a.nchunks - 1;
  const int nlast = a.n - 1;
  const int64_t olast = a.noff > 0 ? a.noff - 1 : 0;
  const int xs = a.nrhs;
  StageB<T> sb{-1, 0, 0};
  MStageC<T, R> sc;
  sc.c = -1;
  sc.meta = 0;
  MStageD<T, R> sd;
  sd.c = -1;
  sd.lg = 0;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    sc.k[u] = -1;
    sc.p0[u] = sc.p1[u] = 0;
    sc.d[u] = T(1);
    sd.k[u] = -1;
#pragma unroll
    for (int q = 0; q < 4; ++q) sd.j[u][q] = -1;
  }
  int t = tb;
  int cur = wlist[tb < te ? tb : llast];
  for (;;) {
    // ---- A: descriptor of a new chunk
    StageB<T> nb{-1, 0, 0};
    {
      const bool live = t < te;
      const int cn = wave_uniform(cur);
      nb.start = cstart[cn];
      nb.meta = cmeta[cn];
      if (live) {
        nb.c = cn;
        ++t;
      }
      cur = wlist[t < te ? t : llast];
    }
    // ---- D (issue): gather x of every row of the chunk whose entries arrived
    const int qd = lane & ((1 << sd.lg) - 1);
    const T* xq = a.xp + (qd < xs ? qd : 0);
    T xv[R][4];
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        xv[u][q] = load_agent(xq + static_cast<int64_t>(sd.j[u][q] >= 0 ? sd.j[u][q] : 0) * xs);
    // ---- B: row bounds and diagonal of the R rows described last time
    MStageC<T, R> nc;
    nc.c = sb.c;
    nc.meta = sb.meta;
    {
      const int lg = sb.meta >> 16, cnt = sb.meta & 0xffff;
      const int g = lane >> lg, groups = 64 >> lg;
      const bool col_ok = (lane & ((1 << lg) - 1)) < a.nrhs;
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int rr = g + groups * u;
        const bool live = sb.c >= 0 && col_ok && rr < cnt;
        const int kk = live ? sb.start + rr : nlast;
        nc.k[u] = live ? kk : -1;
        nc.p0[u] = a.off_ptr[kk];
        nc.p1[u] = a.off_ptr[kk + 1];
        nc.d[u] = a.dinv[kk];
      }
    }
    // ---- C: first four entries and b of the R rows bounded last time
    MStageD<T, R> nd;
    nd.c = sc.c;
    nd.lg = sc.meta >> 16;
    {
      const int gl = lane & ((1 << nd.lg) - 1);
#pragma unroll
      for (int u = 0; u < R; ++u) {
        nd.k[u] = sc.k[u];
        nd.d[u] = sc.d[u];
        nd.e[u] = sc.p0[u];
        nd.e1[u] = sc.p1[u];
        const bool live = sc.c >= 0 && sc.k[u] >= 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ee = nd.e[u] + q;
          const bool ok = live && ee < nd.e1[u];
          const int64_t ec = ok ? ee : olast;
          const int jj = a.off_pos[ec];
          const T vv = a.off_val[ec];
          nd.j[u][q] = ok ? jj : -1;
          nd.v[u][q] = ok ? vv : T(0);
        }
        const T bb = a.bp[live ? static_cast<int64_t>(sc.k[u]) * xs + gl : 0];
        nd.bi[u] = live ? bb : T(0);
      }
    }
    // ---- D (finish): per row, wait, accumulate, rest of the row, publish
    if (sd.c >= 0) {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        if (sd.k[u] < 0) continue;
        wait_values<T, 4>(xq, xs, sd.j[u], xv[u], a.spin_limit, a.status, a.poll != 0);
        T sum = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (sd.j[u][q] >= 0) sum = fma_t(sd.v[u][q], xv[u][q], sum);
        if (sd.e[u] + 4 < sd.e1[u])
          sum = row_dot<T, true>(a.off_pos, a.off_val, sd.e[u] + 4, sd.e1[u], 1, xq, xs,
                                 a.spin_limit, a.status, a.poll != 0, sum);
        const int64_t kq = static_cast<int64_t>(sd.k[u]) * xs;
        store_agent(a.xp + kq + qd, canonical((sd.bi[u] - sum) * sd.d[u]));
        const int KL = 1 << sd.lg;
        for (int q = qd + KL; q < a.nrhs; q += KL) {
          const T s2 = row_dot<T, true>(a.off_pos, a.off_val, sd.e[u], sd.e1[u], 1, a.xp + q, xs,
                                        a.spin_limit, a.status, a.poll != 0, T(0));
          store_agent(a.xp + kq + q, canonical((a.bp[kq + q] - s2) * sd.d[u]));
        }
      }
    } else if (sc.c < 0 && sb.c < 0 && nb.c < 0) {
      return;                         // pipeline drained
    }
    sd = nd;
    sc = nc;
    sb = nb;
  }
}

// ------------------------------- several right-hand sides: layout passes
// The multi-RHS solves work in position order: bp[k * nrhs + q] and xp[k *
// nrhs + q] for the row solved at position k (row_pos is the inverse of
// pos_row).  The caller's B and X are column-major, where the rows of one
// level are scattered (in natural order, consecutive rows sit in consecutive
// levels), so reading B and writing X inside the solve would touch a
// separate cache line per value.  These passes move a tile of 64
// consecutive rows and up to QC columns through LDS instead: down the
// columns of B / X (64 rows contiguous per column) and along the rows of bp
// / xp (the tile's columns contiguous per row).  The tile is only as wide as
// the column count needs (QC = 8, 16, 32 or 64, one padding column against
// bank conflicts), so narrow solves keep many workgroups per CU and enough
// loads in flight to stream at close to the copy rate.
template <typename T, int QC>
__global__ void __launch_bounds__(256)
k_multi_in(int n, int nrhs, int ld, const T* __restrict__ B, const int* __restrict__ row_pos,
           T* __restrict__ bp, T* __restrict__ xp, int fill, int* arrive) {
  using U = typename Bits<T>::U;
  __shared__ T tile[64][QC + 1];
  const int i0 = blockIdx.x * 64, tid = threadIdx.x;
  if (blockIdx.x == 0 && tid == 0) *arrive = 0;
  const int il = tid & 63;
  for (int q0 = 0; q0 < nrhs; q0 += QC) {
    const int qc = nrhs - q0 < QC ? nrhs - q0 : QC;
    if (i0 + il < n)
#pragma unroll
      for (int qq = tid >> 6; qq < QC; qq += 4)
        if (qq < qc) tile[il][qq] = B[static_cast<int64_t>(q0 + qq) * ld + i0 + il];
    __syncthreads();
#pragma unroll
    for (int e = tid; e < 64 * QC; e += 256) {
      const int r = e / qc, qq = e - r * qc;
      if (r < 64 && i0 + r < n) {
        const int64_t o = static_cast<int64_t>(row_pos[i0 + r]) * nrhs + q0 + qq;
        bp[o] = tile[r][qq];
        if (fill) reinterpret_cast<U*>(xp)[o] = Bits<T>::kSentinel;
      }
    }
    __syncthreads();
  }
}

template <typename T, int QC>
__global__ void __launch_bounds__(256)
k_multi_out(int n, int nrhs, int ld, const T* __restrict__ xp, const int* __restrict__ row_pos,
            T* __restrict__ X) {
  __shared__ T tile[64][QC + 1];
  const int i0 = blockIdx.x * 64, tid = threadIdx.x;
  const int il = tid & 63;
  for (int q0 = 0; q0 < nrhs; q0 += QC) {
    const int qc = nrhs - q0 < QC ? nrhs - q0 : QC;
#pragma unroll
    for (int e = tid; e < 64 * QC; e += 256) {
      const int r = e / qc, qq = e - r * qc;
      if (r < 64 && i0 + r < n)
        tile[r][qq] = xp[static_cast<int64_t>(row_pos[i0 + r]) * nrhs + q0 + qq];
    }
    __syncthreads();
    if (i0 + il < n)
#pragma unroll
      for (int qq = tid >> 6; qq < QC; qq += 4)
        if (qq < qc) X[static_cast<int64_t>(q0 + qq) * ld + i0 + il] = tile[il][qq];
    __syncthreads();
  }
}

// row_pos[pos_row[k]] = k
__global__ void __launch_bounds__(256) k_row_pos(int n, const int* __restrict__ pos_row,
                                                 int* __restrict__ row_pos) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) row_pos[pos_row[k]] = k;
}

// ------------------------------------------- block: a workgroup per system
// Level-scheduled inside one workgroup per independent system (block-diagonal
// batches, or one small system): thread t solves row t of each level (and
// t + blockDim, ... for larger levels); the level barrier is a workgroup
// barrier.  kLds: x of the system lives in LDS (the barrier then waits for
// LDS traffic only, so the global loads below stay in flight across it);
// otherwise x is read from the caller's x after a full workgroup barrier.
// Row data of the next two levels are loaded ahead in two raw stages (row
// bounds, then entries and b), as in the static self-scheduled kernel.
// One row per thread, entries in stored order: the arithmetic of the other
// kernels with one lane per row.
template <typename T> struct BlkRow {   // raw row bounds
  int k, p0, p1, i;
  T d;
};
template <typename T> struct BlkEnt {   // raw first entries and b
  int k, e, e1, i;
  T d, bi;
  int j[4];
  T v[4];
};

template <typename T, bool kLds>
__device__ __forceinline__ T blk_x(const T* xs, const T* x, int j, int r0) {
  if constexpr (kLds) return xs[j - r0];
  else return x[j];
}

template <typename T, bool kLds>
__global__ void __launch_bounds__(1024)
k_block(KArgs<T> a, const int* __restrict__ seg_row0, const int* __restrict__ seg_base,
        const int* __restrict__ lev_pos) {
  extern __shared__ __align__(16) unsigned char blk_smem[];
  T* xs = reinterpret_cast<T*>(blk_smem);
  const int s = blockIdx.x;
  const int r0 = seg_row0[s];
  const int lb = seg_base[s];
  const int nl = seg_base[s + 1] - lb - 1;       // levels of this system (-1 if empty)
  const int tid = threadIdx.x, NT = blockDim.x;
  const int nlast = a.n - 1;
  const int64_t olast = a.noff > 0 ? a.noff - 1 : 0;
  auto bounds = [&](int m) {
    BlkRow<T> r{-1, 0, 0, 0, T(1)};
    const int p = (m < nl ? lev_pos[lb + m] : 0) + tid;
    const bool live = m < nl && p < lev_pos[lb + m + 1];
    const int kk = live ? p : nlast;
    r.k = live ? kk : -1;
    r.p0 = a.off_ptr[kk];
    r.p1 = a.off_ptr[kk + 1];
    r.i = a.pos_row[kk];
    r.d = a.dinv[kk];
    return r;
  };
  auto entries = [&](const BlkRow<T>& r) {
    BlkEnt<T> en;
    en.k = r.k;
    en.e = r.p0;
    en.e1 = r.p1;
    en.i = r.i;
    en.d = r.d;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool ok = r.k >= 0 && r.p0 + q < r.p1;
      const int64_t ec = ok ? r.p0 + q : olast;
      const int jj = a.off_col[ec];
      const T vv = a.off_val[ec];
      en.j[q] = ok ? jj : -1;
      en.v[q] = ok ? vv : T(0);
    }
    en.bi = a.b[r.i];
    return en;
  };
  auto finish = [&](int e, int e1, int i, T d, T bi, T sum) {
    for (; e < e1; ++e) sum = fma_t(a.off_val[e], blk_x<T, kLds>(xs, a.x, a.off_col[e], r0), sum);
    const T xi = canonical((bi - sum) * d);
    if constexpr (kLds) xs[i - r0] = xi;
    a.x[i] = xi;
  };
  BlkRow<T> r1 = bounds(1);
  BlkEnt<T> e0 = entries(bounds(0));
  for (int m = 0; m < nl; ++m) {
    const BlkRow<T> r2 = bounds(m + 2);
    const BlkEnt<T> e1 = entries(r1);
    if (e0.k >= 0) {
      T sum = T(0);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (e0.j[q] >= 0) sum = fma_t(e0.v[q], blk_x<T, kLds>(xs, a.x, e0.j[q], r0), sum);
      finish(e0.e + 4, e0.e1, e0.i, e0.d, e0.bi, sum);
    }
    // rows of this level beyond the first blockDim, not loaded ahead
    for (int p = lev_pos[lb + m] + tid + NT; p < lev_pos[lb + m + 1]; p += NT) {
      const int i = a.pos_row[p];
      finish(a.off_ptr[p], a.off_ptr[p + 1], i, a.dinv[p], a.b[i], T(0));
    }
    if constexpr (kLds) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    } else {
      __syncthreads();
    }
    e0 = e1;
    r1 = r2;
  }
}

// ------------------------------------- block, whole system resident in LDS
// The block schedule for systems small enough to live entirely in LDS: the
// workgroup first copies its system's level-ordered data there (values,
// dependency positions and row offsets as 16-bit indices local to the
// system, 1/diagonal, and b, which the solution then overwrites in place:
// row p's b is read only by row p, before its x is stored), then walks the
// levels touching LDS only; x goes to the caller's vector at the end.  A
// lane's row of each level moves through three stages, one level apart, so
// that the loads of a level depend only on values loaded one level earlier
// and a level costs one LDS gather and the row's FMAs:
//   bounds: the row's position, from the level bounds (two levels ahead)
//   row:    its entry range, 1/diagonal and b (one level ahead)
//   entries: its first four dependency positions and values (next level)
// Same arithmetic as every one-lane-per-row solve: entries in stored order,
// FMA from zero, (b - sum) * (1/diagonal).
struct ResBounds {   // bounds stage: raw level bounds
  int m, q0, q1;
};
template <typename T> struct ResRowB {   // row stage: raw
  int m, q0, q1, e, e1;
  T d, bi;
};
template <typename T> struct ResRowC {   // entries stage: raw
  int m, q0, q1, e, e1;
  T d, bi;
  int j[4];
  T v[4];
};

template <typename T>
__global__ void __launch_bounds__(1024)
k_block_res(KArgs<T> a, const int* __restrict__ seg_base, const int* __restrict__ lev_pos) {
  extern __shared__ __align__(16) unsigned char blk_smem[];
  const int lb = seg_base[blockIdx.x];
  const int nl = seg_base[blockIdx.x + 1] - lb - 1;   // levels of this system (-1 if empty)
  if (nl <= 0) return;
  const int tid = threadIdx.x, NT = blockDim.x;
  const int p0 = lev_pos[lb];
  const int ns = lev_pos[lb + nl] - p0;
  const int e0 = a.off_ptr[p0];
  const int ne = a.off_ptr[p0 + ns] - e0;
  // entry ne is a dummy (value -0, dependency: slot ns of xv, which holds
  // +0) that rows with fewer than four entries use for the missing ones
  T* xv = reinterpret_cast<T*>(blk_smem);       // [ns+1] b, then x, by local position
  T* dv = xv + ns + 1;                          // [ns] 1/diagonal
  T* vv = dv + ns;                              // [ne+1] off-diagonal values
  unsigned short* rp = reinterpret_cast<unsigned short*>(vv + ne + 1);   // [ns+1] entry offsets
  unsigned short* cp = rp + ns + 1;             // [ne+1] local position of each dependency
  unsigned short* lp = cp + ne + 1;             // [nl+1] level bounds
  // staging: U rows / entries per thread in flight (clamped in-range indices
  // for the loads of a batch's missing tail, whose results are dropped)
  constexpr int U = 4;
  for (int base = tid; base < ns; base += NT * U) {
    int pr[U], op[U];
    T dd[U], bb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = base + u * NT;
      const int pc = p < ns ? p : ns - 1;
      pr[u] = a.pos_row[p0 + pc];
      dd[u] = a.dinv[p0 + pc];
      op[u] = a.off_ptr[p0 + pc];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) bb[u] = a.b[pr[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = base + u * NT;
      if (p < ns) {
        xv[p] = bb[u];
        dv[p] = dd[u];
        rp[p] = static_cast<unsigned short>(op[u] - e0);
      }
    }
  }
  for (int base = tid; base < ne; base += NT * 2 * U) {
    int cc[2 * U];
    T va[2 * U];
#pragma unroll
    for (int u = 0; u < 2 * U; ++u) {
      const int e = base + u * NT;
      const int ec = e < ne ? e : ne - 1;
      va[u] = a.off_val[e0 + ec];
      cc[u] = a.off_pos[e0 + ec];
    }
#pragma unroll
    for (int u = 0; u < 2 * U; ++u) {
      const int e = base + u * NT;
      if (e < ne) {
        vv[e] = va[u];
        cp[e] = static_cast<unsigned short>(cc[u] - p0);
      }
    }
  }
  for (int m = tid; m <= nl; m += NT) lp[m] = static_cast<unsigned short>(lev_pos[lb + m] - p0);
  if (tid == 0) {
    rp[ns] = static_cast<unsigned short>(ne);
    xv[ns] = T(0);
    vv[ne] = -T(0);
    cp[ne] = static_cast<unsigned short>(ns);
  }
  __syncthreads();
  // Each stage only loads: what it loaded is tested (is there a row, is the
  // entry the row's) one level later, so no stage waits for its own loads.
  // bounds stage: level m's position range (clamped past the last level)
  auto stage_bounds = [&](int m) {
    const int mc = m < nl ? m : nl - 1;
    return ResBounds{m, lp[mc], lp[mc + 1]};
  };
  // this thread's first row of the level, or -1
  auto row_of = [&](int m, int q0, int q1) {
    const int p = q0 + tid;
    return m < nl && p < q1 ? p : -1;
  };
  // row stage (reads b of a row two levels before that row is solved)
  auto stage_row = [&](const ResBounds& bd) {
    const int p = row_of(bd.m, bd.q0, bd.q1);
    const int pc = p >= 0 ? p : 0;
    return ResRowB<T>{bd.m, bd.q0, bd.q1, rp[pc], rp[pc + 1], dv[pc], xv[pc]};
  };
  // entries stage: four loads at once; entries the row lacks (or every
  // entry, if the thread has no row) read the dummy.  Its product is
  // (-0) * (+0) = -0, and s + (-0) == s for every s, zeros of either sign
  // included, so the FMAs of the dummy leave the sum's bits unchanged.
  auto stage_entries = [&](const ResRowB<T>& r) {
    ResRowC<T> c{r.m, r.q0, r.q1, r.e, r.e1, r.d, r.bi, {}, {}};
    const bool live = row_of(r.m, r.q0, r.q1) >= 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ec = live && r.e + q < r.e1 ? r.e + q : ne;
      c.j[q] = cp[ec];
      c.v[q] = vv[ec];
    }
    return c;
  };
  // the levels, walked by the first `nt` threads (one wavefront)
  auto walk = [&](int nt) {
    ResRowC<T> sc = stage_entries(stage_row(stage_bounds(0)));
    ResRowB<T> sb = stage_row(stage_bounds(1));
    ResBounds sa = stage_bounds(2);
    for (int m = 0; m < nl; ++m) {
      // gather of level m first: the stage loads below do not wait for it
      const int p = row_of(sc.m, sc.q0, sc.q1);
      T xg[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) xg[q] = xv[sc.j[q]];
      const ResRowC<T> nc = stage_entries(sb);     // level m+1
      const ResRowB<T> nb = stage_row(sa);         // level m+2 (its b is not written yet)
      const ResBounds na = stage_bounds(m + 3);
      if (p >= 0) {
        T sum = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) sum = fma_t(sc.v[q], xg[q], sum);
        for (int e = sc.e + 4; e < sc.e1; ++e) sum = fma_t(vv[e], xv[cp[e]], sum);
        xv[p] = canonical((sc.bi - sum) * sc.d);
      }
      // rows of this level beyond the first nt, not staged ahead
      for (int r = sc.q0 + tid + nt; r < sc.q1; r += nt) {
        T sum = T(0);
        for (int e = rp[r]; e < rp[r + 1]; ++e) sum = fma_t(vv[e], xv[cp[e]], sum);
        xv[r] = canonical((xv[r] - sum) * dv[r]);
      }
      __builtin_amdgcn_wave_barrier();   // keeps the level's LDS accesses in order
      sc = nc;
      sb = nb;
      sa = na;
    }
  };
  // Wavefront 0 walks the levels with no barrier: the LDS performs one
  // wavefront's accesses in issue order, so a value stored at level m is what
  // a lane of level m+1 reads.  (Rows of a level beyond its 64 lanes are
  // solved one pass after another; the library picks this kernel when every
  // level fits.)  The other wavefronts wait at the barrier below and help with
  // the copy out.
  if (tid < 64) walk(64);
  __syncthreads();
  for (int base = tid; base < ns; base += NT * U) {
    int pr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = base + u * NT;
      pr[u] = a.pos_row[p0 + (p < ns ? p : ns - 1)];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (base + u * NT < ns) a.x[pr[u]] = xv[base + u * NT];
  }
}

// ------------------------------------------------------ self, flag sync
// Rows of a chunk: wait for the flags of all their dependencies, acquire,
// solve reading the caller's x (same per-row order as solve_chunk), release,
// stamp the rows' flags with this solve's epoch.
template <typename T>
__global__ void __launch_bounds__(256) k_self_flag(KArgs<T> a) {
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
    const int cnt = meta & 0xffff, lg = meta >> 16;
    const int G = 1 << lg;
    const int rstep = 64 >> lg;
    const int r0 = lane >> lg, gl = lane & (G - 1);
    for (int rr = r0; rr < cnt; rr += rstep) {
      const int k = start + rr;
      for (int e = a.off_ptr[k] + gl; e < a.off_ptr[k + 1]; e += G) {
        const unsigned* f = a.flags + a.off_col[e];
        if (__hip_atomic_load(const_cast<unsigned*>(f), __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT) != epoch)
          wait_flag(f, epoch, a.spin_limit, a.status);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    for (int rb = 0; rb < cnt; rb += rstep) {     // wave-uniform trip count
      const int rr = rb + r0;
      const bool active = rr < cnt;
      const int k = start + rr;
      T sum = T(0);
      if (active)
        sum = row_dot<T, false>(a.off_col, a.off_val, a.off_ptr[k] + gl, a.off_ptr[k + 1], G, a.x,
                                1, 0, a.status, false, T(0));
      sum = group_sum(sum, lg);
      if (active && gl == 0) {
        const int i = a.pos_row[k];
        a.x[i] = canonical((a.b[i] - sum) * a.dinv[k]);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (gl == 0)
      for (int rr = r0; rr < cnt; rr += rstep)
        __hip_atomic_store(a.flags + a.pos_row[start + rr], epoch, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ------------------------------------------------------------ utilities
template <typename T>
__global__ void __launch_bounds__(256) k_gather(int64_t noff, int n, const int* __restrict__ off_src,
                                                const int* __restrict__ diag_src,
                                                const T* __restrict__ vals, T* __restrict__ off_val,
                                                T* __restrict__ diag, T* __restrict__ dinv,
                                                int* status) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t total = noff > n ? noff : n;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += stride) {
    if (t < noff) off_val[t] = vals[off_src[t]];
    if (t < n) {
      const int s = diag_src[t];
      const T d = s >= 0 ? vals[s] : T(1);
      diag[t] = d;
      dinv[t] = T(1) / d;
      if (d == T(0)) raise_status(status, kStatusZeroPivot);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_fill_sentinel(T* xp, int64_t count, int* arrive) {
  using U = typename Bits<T>::U;
  U* u = reinterpret_cast<U*>(xp);
  if (blockIdx.x == 0 && threadIdx.x == 0) *arrive = 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < count;
       t += stride)
    u[t] = Bits<T>::kSentinel;
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
                                                      unsigned* flags, int* arrive, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    *ticket = 0;
    *status = 0;
    *epoch = 1u;
    *arrive = 0;
  }
  for (int i = t; i < n; i += gridDim.x * blockDim.x) flags[i] = 0u;
}

template <typename T> KArgs<T> make_args(const SolveArgs& s) {
  KArgs<T> a;
  a.chunk_start = s.chunks ? s.chunks->start : nullptr;
  a.chunk_meta = s.chunks ? s.chunks->meta : nullptr;
  a.nchunks = s.chunks ? s.chunks->count : 0;
  a.n = s.plan->n;
  a.noff = s.plan->noff;
  a.off_ptr = s.plan->off_ptr;
  a.off_col = s.plan->off_col;
  a.off_pos = s.plan->off_pos;
  a.off_val = static_cast<const T*>(s.plan->off_val);
  a.dinv = static_cast<const T*>(s.plan->dinv);
  a.pos_row = s.plan->pos_row;
  a.b = static_cast<const T*>(s.b);
  a.x = static_cast<T*>(s.x);
  a.xp = static_cast<T*>(s.xp);
  a.bp = static_cast<const T*>(s.bp);
  a.ld = s.ld;
  a.nrhs = s.nrhs;
  a.ticket = s.scratch.ticket;
  a.status = s.scratch.status;
  a.epoch = s.scratch.epoch;
  a.flags = s.scratch.flags;
  a.arrive = s.scratch.arrive;
  a.res_limit = s.res_limit;
  a.spin_limit = s.spin_limit;
  a.poll = s.poll;
  a.chunk_col = s.chunks ? s.chunks->col : nullptr;
  a.xp_col = s.xp_col;
  return a;
}

inline int blocks_for(int64_t work, int per_block, int cap) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  return static_cast<int>(b < cap ? b : cap);
}

template <typename F> int occupancy(F kernel, int wg) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, wg, 0) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace

template <typename T>
hipError_t launch_gather(const DevPlan& p, const T* vals, int* status, hipStream_t s) {
  const int64_t total = p.noff > p.n ? p.noff : p.n;
  if (total == 0) return hipSuccess;
  k_gather<T><<<blocks_for(total, 256, 65536), 256, 0, s>>>(
      p.noff, p.n, p.off_src, p.diag_src, vals, static_cast<T*>(p.off_val),
      static_cast<T*>(p.diag), static_cast<T*>(p.dinv), status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_sentinel(T* xp, int64_t count, int* arrive, hipStream_t s) {
  k_fill_sentinel<T><<<blocks_for(count, 256, 8192), 256, 0, s>>>(xp, count, arrive);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_multi_in(int n, int nrhs, int ld, const T* B, const int* row_pos, T* bp, T* xp,
                           bool fill, int* arrive, hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  const dim3 grid((n + 63) / 64);
  const int f = fill ? 1 : 0;
  if (nrhs <= 8) k_multi_in<T, 8><<<grid, 256, 0, s>>>(n, nrhs, ld, B, row_pos, bp, xp, f, arrive);
  else if (nrhs <= 16) k_multi_in<T, 16><<<grid, 256, 0, s>>>(n, nrhs, ld, B, row_pos, bp, xp, f, arrive);
  else if (nrhs <= 32) k_multi_in<T, 32><<<grid, 256, 0, s>>>(n, nrhs, ld, B, row_pos, bp, xp, f, arrive);
  else k_multi_in<T, 64><<<grid, 256, 0, s>>>(n, nrhs, ld, B, row_pos, bp, xp, f, arrive);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_multi_out(int n, int nrhs, int ld, const T* xp, const int* row_pos, T* X,
                            hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  const dim3 grid((n + 63) / 64);
  if (nrhs <= 8) k_multi_out<T, 8><<<grid, 256, 0, s>>>(n, nrhs, ld, xp, row_pos, X);
  else if (nrhs <= 16) k_multi_out<T, 16><<<grid, 256, 0, s>>>(n, nrhs, ld, xp, row_pos, X);
  else if (nrhs <= 32) k_multi_out<T, 32><<<grid, 256, 0, s>>>(n, nrhs, ld, xp, row_pos, X);
  else k_multi_out<T, 64><<<grid, 256, 0, s>>>(n, nrhs, ld, xp, row_pos, X);
  return hipGetLastError();
}

hipError_t launch_row_pos(int n, const int* pos_row, int* row_pos, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_row_pos<<<(n + 255) / 256, 256, 0, s>>>(n, pos_row, row_pos);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_level_flat(const SolveArgs& sa, int k0, int k1, hipStream_t s) {
  if (k1 <= k0) return hipSuccess;
  k_level_flat<T><<<blocks_for(k1 - k0, 256, 1 << 30), 256, 0, s>>>(make_args<T>(sa), k0, k1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_level(const SolveArgs& sa, int cb, int ce, hipStream_t s) {
  if (ce <= cb) return hipSuccess;
  const int wpb = sa.wg / 64;
  const int grid = blocks_for(ce - cb, wpb, 1 << 30);
  if (sa.nrhs > 1) k_level<T, true><<<grid, sa.wg, 0, s>>>(make_args<T>(sa), cb, ce);
  else k_level<T, false><<<grid, sa.wg, 0, s>>>(make_args<T>(sa), cb, ce);
  return hipGetLastError();
}

template <typename T> hipError_t launch_self_value(const SolveArgs& sa, hipStream_t s) {
  if (sa.chunks->count == 0) return hipSuccess;
  if (sa.nrhs > 1) k_self_value<T, true><<<sa.grid, sa.wg, 0, s>>>(make_args<T>(sa));
  else k_self_value<T, false><<<sa.grid, sa.wg, 0, s>>>(make_args<T>(sa));
  return hipGetLastError();
}

// the static single-RHS kernel for a slot width (kCols: column-batched table)
template <typename T, bool kCols> const void* static_fn(int stride) {
  return stride == 16  ? reinterpret_cast<const void*>(k_self_static<T, 16, kCols>)
         : stride == 8 ? reinterpret_cast<const void*>(k_self_static<T, 8, kCols>)
         : stride == 4 ? reinterpret_cast<const void*>(k_self_static<T, 4, kCols>)
         : stride == 2 ? reinterpret_cast<const void*>(k_self_static<T, 2, kCols>)
                       : reinterpret_cast<const void*>(k_self_static<T, 1, kCols>);
}

template <typename T> hipError_t launch_self_static(const SolveArgs& sa, hipStream_t s) {
  if (sa.chunks->count == 0) return hipSuccess;
  KArgs<T> ka = make_args<T>(sa);
  const int* cs = sa.chunks->start;
  const int* cm = sa.chunks->meta;
  const int* wp = sa.wave_ptr;
  const int* wl = sa.wave_list;
  void* args[] = {&ka, &cs, &cm, &wp, &wl};
  const void* fn;
  if (sa.nrhs > 1)
    fn = sa.mrows >= 4   ? reinterpret_cast<const void*>(k_self_multi<T, 4>)
         : sa.mrows == 2 ? reinterpret_cast<const void*>(k_self_multi<T, 2>)
                         : reinterpret_cast<const void*>(k_self_multi<T, 1>);
  else
    fn = sa.chunks->col ? static_fn<T, true>(sa.xp_stride) : static_fn<T, false>(sa.xp_stride);
  // the grid's residency is checked by its own wavefronts (grid_resident); a
  // cooperative launch guarantees it up front at a cost of about 16 us
  if (sa.coop) return hipLaunchCooperativeKernel(fn, dim3(sa.grid), dim3(sa.wg), args, 0, s);
  return hipLaunchKernel(fn, dim3(sa.grid), dim3(sa.wg), args, 0, s);
}

template <typename T>
hipError_t launch_block(const SolveArgs& sa, const int* seg_row0, const int* seg_base,
                        const int* lev_pos, int nseg, int threads, int lds_rows, hipStream_t s) {
  if (nseg == 0) return hipSuccess;
  const KArgs<T> ka = make_args<T>(sa);
  if (lds_rows > 0) {
    const size_t bytes = static_cast<size_t>(lds_rows) * sizeof(T);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_block<T, true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(bytes));
    if (e != hipSuccess) return e;
    k_block<T, true><<<nseg, threads, bytes, s>>>(ka, seg_row0, seg_base, lev_pos);
  } else {
    k_block<T, false><<<nseg, threads, 0, s>>>(ka, seg_row0, seg_base, lev_pos);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_block_res(const SolveArgs& sa, const int* seg_base, const int* lev_pos, int nseg,
                           int threads, int lds_bytes, hipStream_t s) {
  if (nseg == 0) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_block_res<T>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (e != hipSuccess) return e;
  k_block_res<T><<<nseg, threads, lds_bytes, s>>>(make_args<T>(sa), seg_base, lev_pos);
  return hipGetLastError();
}

template <typename T> hipError_t launch_self_flag(const SolveArgs& sa, hipStream_t s) {
  if (sa.chunks->count == 0) return hipSuccess;
  k_self_flag<T><<<sa.grid, sa.wg, 0, s>>>(make_args<T>(sa));
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
  k_init_scratch<<<blocks_for(n > 0 ? n : 1, 256, 4096), 256, 0, s>>>(
      sc.ticket, sc.status, sc.epoch, sc.flags, sc.arrive, n);
  return hipGetLastError();
}

// the multi-RHS forms use at least as many registers: size for the smaller
template <typename T> int self_value_blocks_per_cu(int wg) {
  const int a = occupancy(k_self_value<T, false>, wg), b = occupancy(k_self_value<T, true>, wg);
  return a < b ? a : b;
}
template <typename T> int self_flag_blocks_per_cu(int wg) { return occupancy(k_self_flag<T>, wg); }
template <typename T> int self_static_blocks_per_cu(int wg) {
  int m = 1 << 30;
  for (int stride : {1, 2, 4, 8, 16})
    for (const void* fn : {static_fn<T, false>(stride), static_fn<T, true>(stride)})
      m = std::min(m, occupancy(fn, wg));
  return m;
}
template <typename T> int self_multi_blocks_per_cu(int wg, int rows) {
  return rows >= 4   ? occupancy(k_self_multi<T, 4>, wg)
         : rows == 2 ? occupancy(k_self_multi<T, 2>, wg)
                     : occupancy(k_self_multi<T, 1>, wg);
}

#define SPTRSV_INSTANTIATE(T)                                                                    \
  template hipError_t launch_gather<T>(const DevPlan&, const T*, int*, hipStream_t);             \
  template hipError_t launch_fill_sentinel<T>(T*, int64_t, int*, hipStream_t);                   \
  template hipError_t launch_multi_in<T>(int, int, int, const T*, const int*, T*, T*, bool,       \
                                         int*, hipStream_t);                                     \
  template hipError_t launch_multi_out<T>(int, int, int, const T*, const int*, T*, hipStream_t);  \
  template hipError_t launch_level<T>(const SolveArgs&, int, int, hipStream_t);                  \
  template hipError_t launch_self_value<T>(const SolveArgs&, hipStream_t);                       \
  template hipError_t launch_self_flag<T>(const SolveArgs&, hipStream_t);                        \
  template hipError_t launch_self_static<T>(const SolveArgs&, hipStream_t);                      \
  template hipError_t launch_block<T>(const SolveArgs&, const int*, const int*, const int*, int, \
                                      int, int, hipStream_t);                                    \
  template hipError_t launch_level_flat<T>(const SolveArgs&, int, int, hipStream_t);          \
  template hipError_t launch_block_res<T>(const SolveArgs&, const int*, const int*, int, int, int, \
                                          hipStream_t);                                          \
  template hipError_t launch_grad_vals<T>(int, const int*, const int*, int, const T*, const T*,  \
                                          T*, hipStream_t);                                      \
  template int self_value_blocks_per_cu<T>(int);                                                 \
  template int self_flag_blocks_per_cu<T>(int);                                                  \
  template int self_static_blocks_per_cu<T>(int);                                                \
  template int self_multi_blocks_per_cu<T>(int, int);

SPTRSV_INSTANTIATE(double)
SPTRSV_INSTANTIATE(float)

}  // namespace sptrsv
