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

#include "analysis.hpp"
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
  int n;
  int64_t noff;
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

// Continues `sum` over the lane's entries e, e+G, e+2G, ... < e1 of one row,
// four entries in flight at a time.  kPoll: x is read with agent-scope atomic
// loads and sentinel values are waited for.
template <typename T, bool kPoll>
__device__ __forceinline__ T row_dot(const int* __restrict__ off_col,
                                     const T* __restrict__ off_val, int e, int e1, int G,
                                     const T* x, int spin_limit, int* status, T sum) {
  for (; e < e1; e += 4 * G) {
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

template <typename T, bool kPoll> __device__ __forceinline__ void store_x(T* p, T v) {
  if constexpr (kPoll) store_agent(p, v);
  else *p = v;
}

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Solves the rows of one chunk (see the chunk encoding in analysis.hpp).
//  G = 1: lane l owns rows start+l, start+l+64, ... (up to kMaxRowsPerLane);
//         the bounds, first four entries, x gathers, b and diagonal of all its
//         rows are issued before any wait, then each row is finished.
//  G > 1: rows of G lanes; lanes stride the row, the group sums by butterfly.
// Per row the accumulation order is the same in every kernel using this, so
// level- and self-scheduled solves agree bit for bit at equal chunking.
template <typename T, bool kPoll>
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
        di[u] = a.diag[k[u]];
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
        j[u][q] = ee < e1[u] ? a.off_col[ee] : -1;
        v[u][q] = ee < e1[u] ? a.off_val[ee] : T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
      for (int q = 0; q < E; ++q)
        xv[u][q] = j[u][q] >= 0 ? (kPoll ? load_agent(a.x + j[u][q]) : a.x[j[u][q]]) : T(0);
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (k[u] < 0) continue;
      T sum = T(0);
#pragma unroll
      for (int q = 0; q < E; ++q) {
        if (j[u][q] < 0) continue;
        T xx = xv[u][q];
        if (kPoll && is_sentinel(xx)) xx = wait_value(a.x + j[u][q], a.spin_limit, a.status);
        sum = __builtin_fma(v[u][q], xx, sum);
      }
      if (e1[u] > e0[u] + E)
        sum = row_dot<T, kPoll>(a.off_col, a.off_val, e0[u] + E, e1[u], 1, a.x, a.spin_limit,
                                a.status, sum);
      store_x<T, kPoll>(a.x + i[u], canonical((bi[u] - sum) / di[u]));
    }
    return;
  }
  const int r = lane >> lg, gl = lane & ((1 << lg) - 1);
  const bool active = r < cnt;
  const int k = start + r;
  T sum = T(0);
  if (active)
    sum = row_dot<T, kPoll>(a.off_col, a.off_val, a.off_ptr[k] + gl, a.off_ptr[k + 1], 1 << lg,
                            a.x, a.spin_limit, a.status, T(0));
  sum = group_sum(sum, lg);
  if (active && gl == 0) {
    const int i = a.pos_row[k];
    store_x<T, kPoll>(a.x + i, canonical((a.b[i] - sum) / a.diag[k]));
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
template <typename T>
__global__ void __launch_bounds__(256) k_level(KArgs<T> a, int chunk_begin, int chunk_end) {
  const int lane = threadIdx.x & 63;
  const int c = wave_uniform(chunk_begin + static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  if (c >= chunk_end) return;
  solve_chunk<T, false>(a, a.chunk_start[c], a.chunk_meta[c], lane);
}

// ----------------------------------------------------- self, value sync
template <typename T>
__global__ void __launch_bounds__(256) k_self_value(KArgs<T> a) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    const int c = claim_chunk(a.ticket, a.nchunks, lane);
    if (c < 0) return;
    solve_chunk<T, true>(a, a.chunk_start[c], a.chunk_meta[c], lane);
  }
}

// ------------------------------------- self, value sync, static pipeline
// Wavefront w of W takes chunks w, w+W, w+2W, ... in that order (the grid is
// launched cooperatively, so all W wavefronts are resident: the wavefront
// holding the lowest unfinished chunk has finished its earlier chunks and is
// working on it, and that chunk's dependencies are done).  No claim atomics.
// Each chunk moves through four stages, one chunk apart, so the dependent
// index loads of later chunks are in flight while this one waits on x:
//   A descriptor -> B row bounds, row, diagonal -> C first entries, b
//   -> D gather x (poll), accumulate, store.
// Per row the arithmetic is that of solve_chunk with one row per lane.
// Each stage only stores raw loaded values; any arithmetic on them happens
// one iteration later, so no wait for a load is needed before the next
// stage's loads (and the x gathers) have been issued.
template <typename T> struct StageB {   // descriptor, raw
  int c, start, meta;
};
template <typename T> struct StageC {   // row bounds, raw
  int c, meta, k, p0, p1, i;
  T d;
};
template <typename T> struct StageD {   // first entries of the lane, raw
  int c, lg, k, e, e1, i;
  T d, bi;
  int j[4];
  T v[4];
};

// kMulti: several right-hand sides (column stride ld).  The lanes of a row
// take columns q0 = lane % KL (KL = 2^lg lanes per row) instead of entries;
// every lane walks all entries of its row in order, so each column is solved
// exactly as the single right-hand side with one lane per row.  Columns
// beyond the first KL are finished by the same lanes, unpipelined.
template <typename T, bool kMulti>
__global__ void __launch_bounds__(256)
k_self_static(KArgs<T> a, const int* __restrict__ cstart, const int* __restrict__ cmeta) {
  const int lane = threadIdx.x & 63;
  const int W = static_cast<int>(gridDim.x * (blockDim.x >> 6));
  const int w = wave_uniform(static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const int nch = a.nchunks;
  const int nlast = a.n - 1;          // clamp for loads whose result is discarded
  const int64_t olast = a.noff > 0 ? a.noff - 1 : 0;
  StageB<T> sb{-1, 0, 0};
  StageC<T> sc{-1, 0, -1, 0, 0, 0, T(1)};
  StageD<T> sd;
  sd.c = -1;
  sd.lg = 0;
  sd.k = -1;
#pragma unroll
  for (int q = 0; q < 4; ++q) sd.j[q] = -1;
  int next = w;                       // next chunk to enter stage A
  for (;;) {
    // ---- A: descriptor of a new chunk (uniform index, read-only table)
    StageB<T> nb{-1, 0, 0};
    {
      const int cn = wave_uniform(next < nch ? next : nch - 1);
      nb.start = cstart[cn];
      nb.meta = cmeta[cn];
      if (next < nch) {
        nb.c = next;
        next += W;
      }
    }
    // ---- D (issue): gather x for the chunk whose entries arrived last time
    const int64_t xoff_d = kMulti ? static_cast<int64_t>(lane & ((1 << sd.lg) - 1)) * a.ld : 0;
    T xv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      xv[q] = load_agent(a.x + (sd.j[q] >= 0 ? xoff_d + sd.j[q] : 0));
    // ---- B: row bounds, row and diagonal of the chunk described last time
    StageC<T> nc{sb.c, sb.meta, -1, 0, 0, 0, T(1)};
    {
      const int lg = sb.meta >> 16, cnt = sb.meta & 0xffff;
      const int r = lane >> lg;
      bool live = sb.c >= 0 && r < cnt;
      if (kMulti) live = live && (lane & ((1 << lg) - 1)) < a.nrhs;
      const int kk = live ? sb.start + r : nlast;
      nc.k = live ? kk : -1;
      nc.p0 = a.off_ptr[kk];
      nc.p1 = a.off_ptr[kk + 1];
      nc.i = a.pos_row[kk];
      nc.d = a.diag[kk];
    }
    // ---- C: the lane's first four entries and b of the chunk bounded last time
    StageD<T> nd;
    nd.c = sc.c;
    nd.lg = sc.meta >> 16;
    nd.k = sc.k;
    nd.i = sc.i;
    nd.d = sc.d;
    {
      const int G = kMulti ? 1 : 1 << nd.lg;          // entry stride of the lane
      const int gl = lane & ((1 << nd.lg) - 1);
      nd.e = sc.p0 + (kMulti ? 0 : gl);
      nd.e1 = sc.p1;
      const bool live = sc.c >= 0 && sc.k >= 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ee = nd.e + q * G;
        const bool ok = live && ee < nd.e1;
        const int64_t ec = ok ? ee : olast;
        const int jj = a.off_col[ec];
        const T vv = a.off_val[ec];
        nd.j[q] = ok ? jj : -1;
        nd.v[q] = ok ? vv : T(0);
      }
      const int64_t boff = kMulti && live ? static_cast<int64_t>(gl) * a.ld : 0;
      const T bb = a.b[boff + sc.i];
      nd.bi = (live && (kMulti || gl == 0)) ? bb : T(0);
    }
    // ---- D (finish): wait, accumulate, rest of the row, group sum, store
    if (sd.c >= 0) {
      const int G = kMulti ? 1 : 1 << sd.lg;
      T* xq = a.x + xoff_d;
      T sum = T(0);
      if (sd.k >= 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (sd.j[q] < 0) continue;
          T xx = xv[q];
          if (is_sentinel(xx)) xx = wait_value(xq + sd.j[q], a.spin_limit, a.status);
          sum = __builtin_fma(sd.v[q], xx, sum);
        }
        if (sd.e + 4 * G < sd.e1)
          sum = row_dot<T, true>(a.off_col, a.off_val, sd.e + 4 * G, sd.e1, G, xq, a.spin_limit,
                                 a.status, sum);
      }
      if constexpr (kMulti) {
        if (sd.k >= 0) {
          store_agent(xq + sd.i, canonical((sd.bi - sum) / sd.d));
          // columns beyond the first 2^lg, same lane, unpipelined
          const int KL = 1 << sd.lg;
          for (int q = (lane & (KL - 1)) + KL; q < a.nrhs; q += KL) {
            const int64_t off = static_cast<int64_t>(q) * a.ld;
            const T s2 = row_dot<T, true>(a.off_col, a.off_val, sd.e, sd.e1, 1, a.x + off,
                                          a.spin_limit, a.status, T(0));
            store_agent(a.x + off + sd.i, canonical((a.b[off + sd.i] - s2) / sd.d));
          }
        }
      } else {
        sum = group_sum(sum, sd.lg);
        if (sd.k >= 0 && (lane & (G - 1)) == 0)
          store_agent(a.x + sd.i, canonical((sd.bi - sum) / sd.d));
      }
    } else if (sc.c < 0 && sb.c < 0 && nb.c < 0) {
      return;                         // pipeline drained
    }
    sd = nd;
    sc = nc;
    sb = nb;
  }
}

// ------------------------------------------- block: a workgroup per system
// Level-scheduled inside one workgroup per independent system (block-diagonal
// batches, or one small system): thread t solves row t of each level (and
// t + blockDim, ... for larger levels); the level barrier is a workgroup
// barrier.  kLds: x of the system lives in LDS (the barrier then waits for
// LDS traffic only, so the global loads below stay in flight across it);
// otherwise x is read from global memory after a full workgroup barrier.
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
    r.d = a.diag[kk];
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
    for (; e < e1; ++e) sum = __builtin_fma(a.off_val[e], blk_x<T, kLds>(xs, a.x, a.off_col[e], r0), sum);
    const T xi = canonical((bi - sum) / d);
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
        if (e0.j[q] >= 0) sum = __builtin_fma(e0.v[q], blk_x<T, kLds>(xs, a.x, e0.j[q], r0), sum);
      finish(e0.e + 4, e0.e1, e0.i, e0.d, e0.bi, sum);
    }
    // rows of this level beyond the first blockDim, not loaded ahead
    for (int p = lev_pos[lb + m] + tid + NT; p < lev_pos[lb + m + 1]; p += NT) {
      const int i = a.pos_row[p];
      finish(a.off_ptr[p], a.off_ptr[p + 1], i, a.diag[p], a.b[i], T(0));
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

// ------------------------------------------------------ self, flag sync
// Rows of a chunk: wait for the flags of all their dependencies, acquire,
// solve with plain loads (same per-row order as solve_chunk), release, stamp
// the rows' flags with this solve's epoch.
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
                                0, a.status, T(0));
      sum = group_sum(sum, lg);
      if (active && gl == 0) {
        const int i = a.pos_row[k];
        a.x[i] = canonical((a.b[i] - sum) / a.diag[k]);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (gl == 0)
      for (int rr = r0; rr < cnt; rr += rstep)
        __hip_atomic_store(a.flags + a.pos_row[start + rr], epoch, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
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
  const int cnt = meta & 0xffff, lg = meta >> 16;
  const int r = lane >> lg, q0 = lane & ((1 << lg) - 1);
  if (r >= cnt) return;
  const int k = start + r;
  const int i = a.pos_row[k];
  const int e0 = a.off_ptr[k], e1 = a.off_ptr[k + 1];
  const T d = a.diag[k];
  for (int q = q0; q < a.nrhs; q += (1 << lg)) {
    const size_t off = static_cast<size_t>(q) * a.ld;
    const T sum = row_dot<T, kPoll>(a.off_col, a.off_val, e0, e1, 1, a.x + off, a.spin_limit,
                                    a.status, T(0));
    const T xi = canonical((a.b[off + i] - sum) / d);
    if (kPoll) store_agent(a.x + off + i, xi);
    else a.x[off + i] = xi;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_level_multi(KArgs<T> a, int chunk_begin, int chunk_end) {
  const int lane = threadIdx.x & 63;
  const int c = wave_uniform(chunk_begin + static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  if (c >= chunk_end) return;
  multi_rows<T, false>(a, c, lane);
}

template <typename T>
__global__ void __launch_bounds__(256) k_self_multi_value(KArgs<T> a) {
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
  a.n = s.plan->n;
  a.noff = s.plan->noff;
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

template <typename T> hipError_t launch_self_static(const SolveArgs& sa, hipStream_t s) {
  if (sa.chunks->count == 0) return hipSuccess;
  KArgs<T> ka = make_args<T>(sa);
  const int* cs = sa.chunks->start;
  const int* cm = sa.chunks->meta;
  void* args[] = {&ka, &cs, &cm};
  const void* fn = sa.nrhs > 1 ? reinterpret_cast<const void*>(k_self_static<T, true>)
                               : reinterpret_cast<const void*>(k_self_static<T, false>);
  return hipLaunchCooperativeKernel(fn, dim3(sa.grid), dim3(sa.wg), args, 0, s);
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
template <typename T> int self_static_blocks_per_cu(int wg) {
  int nb = 0;
  // the multi-RHS form uses at least as many registers: size for the larger
  int nb1 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_self_static<T, false>, wg, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb1, k_self_static<T, true>, wg, 0) != hipSuccess)
    return 1;
  nb = nb < nb1 ? nb : nb1;
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
  template hipError_t launch_self_static<T>(const SolveArgs&, hipStream_t);                     \
  template hipError_t launch_block<T>(const SolveArgs&, const int*, const int*, const int*, int,   \
                                      int, int, hipStream_t);                                     \
  template int self_static_blocks_per_cu<T>(int);                                               \
  template hipError_t launch_self_multi_value<T>(const SolveArgs&, hipStream_t);                \
  template hipError_t launch_grad_vals<T>(int, const int*, const int*, int, const T*, const T*, \
                                          T*, hipStream_t);                                     \
  template int self_value_blocks_per_cu<T>(int);                                                \
  template int self_flag_blocks_per_cu<T>(int);                                                 \
  template int self_multi_blocks_per_cu<T>(int);

SPTRSV_INSTANTIATE(double)
SPTRSV_INSTANTIATE(float)

}  // namespace sptrsv
