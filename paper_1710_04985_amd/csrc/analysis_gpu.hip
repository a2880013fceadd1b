// Device-side setup phase: validity check, levels, level-ordered layout.
// Section references are to Li, arXiv:1710.04985.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>

#include "analysis.hpp"
#include "analysis_gpu.hpp"

namespace sptrsv {
namespace {

enum : int { kFlagBad = 1, kFlagUnsorted = 2, kFlagTimeout = 4 };

__device__ __forceinline__ int bitlen(unsigned v) { return v ? 32 - __builtin_clz(v) : 0; }

// One row per thread: bounds, column range and side, strictly increasing
// columns, one diagonal (unless unit), dependency count.  Any irregularity
// only raises a flag; the host analysis then decides the exact error.
__global__ void __launch_bounds__(256) k_check(int n, int64_t nnz, const int* __restrict__ rp,
                                               const int* __restrict__ col, int upper, int unit,
                                               int* __restrict__ depcnt, int* flags, int* maxlen) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int f = 0, ml = 0;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += stride) {
    const int i = static_cast<int>(t);
    const int a = rp[i], b = rp[i + 1];
    depcnt[i] = 0;
    if (a < 0 || b < a || b > nnz) {
      f |= kFlagBad;
      continue;
    }
    int nd = 0, dep = 0, prev = -1;
    for (int e = a; e < b; ++e) {
      const int j = col[e];
      if (j < 0 || j >= n) {
        f |= kFlagBad;
        break;
      }
      if (upper ? j < i : j > i) f |= kFlagBad;
      if (e > a && j <= prev) f |= kFlagUnsorted;
      prev = j;
      if (j == i) ++nd;
      else ++dep;
    }
    if (nd > 1 || (!unit && nd != 1)) f |= kFlagBad;
    depcnt[i] = dep;
    ml = dep > ml ? dep : ml;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (rp[0] != 0 || rp[n] != nnz)) f |= kFlagBad;
  if (f) atomicOr(flags, f);
  if (ml) atomicMax(maxlen, ml);
}

__global__ void __launch_bounds__(256) k_fill_int(int* p, int64_t count, int v) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < count; t += stride)
    p[t] = v;
}

// Levels of Sec. 4.1 (0-based), computed without global synchronisation: the
// self-scheduled sweep with max(level)+1 in place of the dot product.  Rows
// are taken in dependency order (ascending for lower, descending for upper)
// in chunks of 64, one row per lane; each workgroup (one wavefront) claims
// the next chunk from a ticket, so chunks are taken in order by running
// wavefronts and no co-residency is assumed.
// level[] starts at -1; a row publishes its level with one agent-scope atomic
// store.  Rows are sorted on this route, so a row's dependencies inside the
// chunk are the off-diagonals next to its diagonal and those in earlier
// chunks one contiguous range.  A round polls the earlier-chunk range
// (sixteen loads in flight, resuming at the first one not yet published),
// then resolves the chain inside the chunk through LDS, one link per step.
// A lane keeps up to kInChunk in-chunk dependencies (6-bit lane numbers)
// packed in a register and rescans its in-chunk range otherwise.  The lowest
// unfinished row always has every dependency published and its chunk held by
// a running wavefront, so the sweep progresses.
constexpr int kInChunk = 10;

__global__ void __launch_bounds__(64)
k_levels(int n, const int* __restrict__ rp, const int* __restrict__ col, int upper,
         int* level, int* flags, int* maxlev, int* ticket, int spin_limit) {
  __shared__ int sl[64];
  const int lane = threadIdx.x;
  const int nch = (n + 63) / 64;
  int wmax = -1;
  for (;;) {
    int c = 0;
    if (lane == 0) c = atomicAdd(ticket, 1);
    c = __builtin_amdgcn_readfirstlane(c);
    if (c >= nch) break;
    const int c0 = c * 64;            // dependency-order index of lane 0
    const int r = c0 + lane;
    const bool live = r < n;
    const int i = live ? (upper ? n - 1 - r : r) : 0;
    const int a = live ? rp[i] : 0, e1 = live ? rp[i + 1] : 0;
    // Rows are sorted on this route (k_check): the in-chunk dependencies are
    // the off-diagonals next to the diagonal, those in earlier chunks the
    // contiguous range [oa, ob)
    unsigned long long pk = 0;
    int nin = 0, oa = a, ob = a, ib = a, ie = a;
    if (live) {
      if (!upper) {
        int e = e1;
        if (e > a && col[e - 1] == i) --e;          // diagonal last
        ie = e;
        while (e > a && col[e - 1] >= c0) {         // in-chunk: c0 <= j < i
          if (nin < kInChunk) pk |= static_cast<unsigned long long>(col[e - 1] - c0) << (6 * nin);
          ++nin;
          --e;
        }
        ib = e;
        oa = a;
        ob = e;
      } else {
        int e = a;
        if (e < e1 && col[e] == i) ++e;             // diagonal first
        ib = e;
        const int jmax = n - 1 - c0;                // in-chunk: i < j <= n-1-c0
        while (e < e1 && col[e] <= jmax) {
          if (nin < kInChunk)
            pk |= static_cast<unsigned long long>(n - 1 - col[e] - c0) << (6 * nin);
          ++nin;
          ++e;
        }
        ie = e;
        oa = e;
        ob = e1;
      }
    }
    int e = oa;                       // cursor over the earlier-chunk dependencies
    int lvl = 0;
    bool done = !live;
    sl[lane] = -1;
    for (int round = 0;; ++round) {
      bool gready = true;
      if (!done) {
        // sixteen at a time: their columns, then their levels, in flight together
        while (e < ob) {
          int v16[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int j = e + q < ob ? col[e + q] : -1;
            v16[q] = j >= 0 ? __hip_atomic_load(level + j, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT)
                            : 0;
          }
          int adv = 0;
          bool stop = false;
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            if (stop || e + q >= ob) continue;
            if (v16[q] < 0) {
              stop = true;
            } else {
              lvl = v16[q] + 1 > lvl ? v16[q] + 1 : lvl;
              ++adv;
            }
          }
          e += adv;
          if (stop) {
            gready = false;
            break;
          }
        }
      }
      for (int step = 0; step < 65; ++step) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        bool progressed = false;
        if (!done && gready) {
          int l2 = lvl;
          bool ready = true;
          if (nin <= kInChunk) {
            for (int q = 0; q < nin; ++q) {
              const int v = sl[(pk >> (6 * q)) & 63];
              if (v < 0) {
                ready = false;
                break;
              }
              l2 = v + 1 > l2 ? v + 1 : l2;
            }
          } else {
            for (int e2 = ib; e2 < ie; ++e2) {
              const int rj = upper ? n - 1 - col[e2] : col[e2];
              const int v = sl[rj - c0];
              if (v < 0) {
                ready = false;
                break;
              }
              l2 = v + 1 > l2 ? v + 1 : l2;
            }
          }
          if (ready) {
            __hip_atomic_store(level + i, l2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sl[lane] = l2;
            wmax = l2 > wmax ? l2 : wmax;
            done = true;
            progressed = true;
          }
        }
        if (!__any(progressed)) break;
      }
      if (__all(done)) break;
      if (round >= spin_limit) {     // cannot happen on a valid triangle: drain
        if (!done) {
          __hip_atomic_store(level + i, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          done = true;
        }
        if (lane == 0) atomicOr(flags, kFlagTimeout);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const int v = __shfl_xor(wmax, o, 64);
    wmax = v > wmax ? v : wmax;
  }
  if (lane == 0 && wmax >= 0) atomicMax(maxlev, wmax);
}

// sort keys: (level, bit length of the dependency count), values: row
__global__ void __launch_bounds__(256) k_keys(int n, const int* __restrict__ level,
                                              const int* __restrict__ depcnt,
                                              unsigned long long* __restrict__ key, int* __restrict__ rows,
                                              unsigned* __restrict__ lkey, int* __restrict__ rows2) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += stride) {
    const int i = static_cast<int>(t);
    key[i] = (static_cast<unsigned long long>(level[i]) << 5) | bitlen(static_cast<unsigned>(depcnt[i]));
    rows[i] = i;
    lkey[i] = static_cast<unsigned>(level[i]);
    rows2[i] = i;
  }
}

// inverse permutation, row length per position, level pointers
__global__ void __launch_bounds__(256) k_positions(int n, int nlev, const int* __restrict__ pos_row,
                                                   const int* __restrict__ level,
                                                   const int* __restrict__ depcnt,
                                                   int* __restrict__ pos_of, int* __restrict__ cnt,
                                                   int* __restrict__ ilev) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t <= n; t += stride) {
    const int k = static_cast<int>(t);
    if (k == n) {
      cnt[n] = 0;
      ilev[nlev] = n;
      continue;
    }
    const int i = pos_row[k];
    pos_of[i] = k;
    cnt[k] = depcnt[i];
    const int lk = level[i];
    if (k == 0 || level[pos_row[k - 1]] != lk) ilev[lk] = k;
  }
}

// off-diagonal entries of each position, in stored order
__global__ void __launch_bounds__(256) k_offdiag(int n, int unit, const int* __restrict__ rp,
                                                 const int* __restrict__ col,
                                                 const int* __restrict__ pos_row,
                                                 const int* __restrict__ pos_of,
                                                 const int* __restrict__ off_ptr,
                                                 int* __restrict__ off_col, int* __restrict__ off_pos,
                                                 int* __restrict__ off_src, int* __restrict__ diag_src) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += stride) {
    const int k = static_cast<int>(t);
    const int i = pos_row[k];
    int o = off_ptr[k];
    int ds = -1;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      const int j = col[e];
      if (j == i) {
        if (!unit) ds = e;
        continue;
      }
      off_col[o] = j;
      off_pos[o] = pos_of[j];
      off_src[o] = e;
      ++o;
    }
    diag_src[k] = ds;
  }
}

inline int blocks(int64_t work) {
  int64_t b = (work + 255) / 256;
  if (b < 1) b = 1;
  return static_cast<int>(b < 65536 ? b : 65536);
}

template <typename T> int dmalloc(T** p, int64_t count) {
  *p = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(p), static_cast<size_t>(count > 0 ? count : 1) * sizeof(T)) !=
      hipSuccess)
    return kErrOom;
  return kOk;
}

struct Temps {
  int* flags = nullptr;
  int* counters = nullptr;   // [0] max row length, [1] max level, [2] chunk ticket
  unsigned long long* key = nullptr;
  unsigned long long* key_s = nullptr;
  int* rows = nullptr;
  unsigned* lkey = nullptr;
  unsigned* lkey_s = nullptr;
  int* rows2 = nullptr;
  int* pos_of = nullptr;
  int* cnt = nullptr;
  int* ilev = nullptr;
  void* tmp = nullptr;
  ~Temps() {
    for (void* p : {static_cast<void*>(flags), static_cast<void*>(counters), static_cast<void*>(key),
                    static_cast<void*>(key_s), static_cast<void*>(rows), static_cast<void*>(lkey),
                    static_cast<void*>(lkey_s), static_cast<void*>(rows2), static_cast<void*>(pos_of),
                    static_cast<void*>(cnt), static_cast<void*>(ilev), tmp})
      if (p) (void)hipFree(p);
  }
};

__global__ void __launch_bounds__(256) k_fill_iota(int* p, int64_t count) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < count; t += stride)
    p[t] = static_cast<int>(t);
}

// row_of[e] = the row of entry e
__global__ void __launch_bounds__(256) k_row_of(int n, const int* __restrict__ rp,
                                                int* __restrict__ row_of) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += stride) {
    const int i = static_cast<int>(t);
    for (int e = rp[i]; e < rp[i + 1]; ++e) row_of[e] = i;
  }
}

// entries of T^T (sorted by (column of T, entry)): column = row of T, source
// = entry of T; row pointers of T^T from the first entry of each column
__global__ void __launch_bounds__(256) k_transpose_fill(int n, int64_t nnz,
                                                        const int* __restrict__ col_sorted,
                                                        const int* __restrict__ src_sorted,
                                                        const int* __restrict__ row_of,
                                                        int* __restrict__ colT, int* __restrict__ rpT) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < nnz; t += stride) {
    colT[t] = row_of[src_sorted[t]];
    // the first entry of column c (and of every empty column before it)
    const int c = col_sorted[t];
    const int cprev = t > 0 ? col_sorted[t - 1] : -1;
    for (int j = cprev + 1; j <= c; ++j) rpT[j] = static_cast<int>(t);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int clast = nnz > 0 ? col_sorted[nnz - 1] : -1;
    for (int j = clast + 1; j <= n; ++j) rpT[j] = static_cast<int>(nnz);
  }
}

// loc[e] = where entry e of the caller's T sits in the forward plan's value
// buffer (off-diagonals, then the diagonal)
__global__ void __launch_bounds__(256) k_value_loc(int n, int64_t noff, const int* __restrict__ off_src,
                                                   const int* __restrict__ diag_src,
                                                   int* __restrict__ loc) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t total = noff > n ? noff : n;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) {
    if (t < noff) loc[off_src[t]] = static_cast<int>(t);
    if (t < n && diag_src[t] >= 0) loc[diag_src[t]] = static_cast<int>(noff + t);
  }
}

// value sources of the T^T plan: entries of T^T -> entries of T -> value
// buffer of the forward plan
__global__ void __launch_bounds__(256) k_compose_src(int n, int64_t noff, const int* __restrict__ srcT,
                                                     const int* __restrict__ loc,
                                                     int* __restrict__ off_src,
                                                     int* __restrict__ diag_src) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t total = noff > n ? noff : n;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) {
    if (t < noff) off_src[t] = loc[srcT[off_src[t]]];
    if (t < n && diag_src[t] >= 0) diag_src[t] = loc[srcT[diag_src[t]]];
  }
}

// block-diagonal concatenation of `count` systems (one row of the grid per
// system): row pointers and columns shifted by the systems before, values
// copied; a column outside its own system, or row pointers that do not run
// from 0 to the system's nnz, raise the flag
struct SysDesc {
  const int* rp;
  const int* col;
  const void* vals;
  int n;
  int nnz;
  int roff;
  int eoff;
};

__global__ void __launch_bounds__(256) k_concat(const SysDesc* __restrict__ sys, int vb,
                                                int* __restrict__ rp_cat, int* __restrict__ col_cat,
                                                unsigned char* __restrict__ vals_cat, int* flags) {
  const SysDesc d = sys[blockIdx.y];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int f = 0;
  const int64_t total = d.nnz > d.n ? d.nnz : d.n;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) {
    if (t < d.n) rp_cat[d.roff + t] = d.rp[t] + d.eoff;
    if (t < d.nnz) {
      const int j = d.col[t];
      if (j < 0 || j >= d.n) f = 1;
      col_cat[d.eoff + t] = j + d.roff;
      if (vb == 8)
        reinterpret_cast<unsigned long long*>(vals_cat)[d.eoff + t] =
            static_cast<const unsigned long long*>(d.vals)[t];
      else
        reinterpret_cast<unsigned*>(vals_cat)[d.eoff + t] = static_cast<const unsigned*>(d.vals)[t];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (d.rp[0] != 0 || d.rp[d.n] != d.nnz)) f = 1;
  if (f) atomicOr(flags, 1);
}

}  // namespace

void free_device_analysis(DeviceAnalysis& a) {
  for (int* p : {a.level, a.depcnt, a.jlev, a.pos_row, a.off_ptr, a.off_col, a.off_pos, a.off_src,
                 a.diag_src})
    if (p) (void)hipFree(p);
  a = DeviceAnalysis();
}

#define DCHK(expr)                                  \
  do {                                              \
    if ((expr) != hipSuccess) {                     \
      free_device_analysis(out);                    \
      return kErrHip;                               \
    }                                               \
  } while (0)
#define DALLOC(ptr, count)                          \
  do {                                              \
    if (dmalloc(&(ptr), (count)) != kOk) {          \
      free_device_analysis(out);                    \
      return kErrOom;                               \
    }                                               \
  } while (0)

int device_analysis(int n, int64_t nnz, const int* row_ptr, const int* col, bool upper,
                    bool unit_diag, int num_cu, hipStream_t s, DeviceAnalysis& out) {
  out = DeviceAnalysis();
  if (n < 1 || nnz < 0 || nnz > INT32_MAX || n > (1 << 30)) return kErrNotSupported;
  out.n = n;
  Temps tp;
  DALLOC(tp.flags, 1);
  DALLOC(tp.counters, 3);
  DALLOC(out.depcnt, n);
  DALLOC(out.level, n);
  int zero2[3] = {0, -1, 0};
  int zero = 0;
  DCHK(hipMemcpyAsync(tp.flags, &zero, sizeof(int), hipMemcpyHostToDevice, s));
  DCHK(hipMemcpyAsync(tp.counters, zero2, 3 * sizeof(int), hipMemcpyHostToDevice, s));
  k_check<<<blocks(n), 256, 0, s>>>(n, nnz, row_ptr, col, upper, unit_diag, out.depcnt, tp.flags,
                                     tp.counters);
  DCHK(hipGetLastError());
  int flags = 0, max_len = 0;
  DCHK(hipMemcpyAsync(&flags, tp.flags, sizeof(int), hipMemcpyDeviceToHost, s));
  DCHK(hipMemcpyAsync(&max_len, tp.counters, sizeof(int), hipMemcpyDeviceToHost, s));
  DCHK(hipStreamSynchronize(s));
  if (flags) {
    free_device_analysis(out);
    return kErrNotSupported;
  }

  // levels
  k_fill_int<<<blocks(n), 256, 0, s>>>(out.level, n, -1);
  DCHK(hipGetLastError());
  {
    int per_cu = 0;
    DCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_levels, 64, 0));
    const int nch = (n + 63) / 64;
    // A waiting lane rereads up to sixteen dependencies per round, so rows
    // longer than that multiply the polling traffic of every wavefront that
    // waits ahead of the level front.  With such rows four wavefronts per CU
    // are used (random power-law triangle: 24 -> 14 ms), otherwise every
    // resident one (mesh triangles, whose level front spans all rows: 6.8 ms,
    // 12.6 ms at four per CU).
    const int waves_per_cu = max_len > 16 ? std::min(4, std::max(1, per_cu)) : std::max(1, per_cu);
    const int grid = std::max(1, std::min(nch, waves_per_cu * num_cu));
    k_levels<<<grid, 64, 0, s>>>(n, row_ptr, col, upper ? 1 : 0, out.level, tp.flags,
                                 tp.counters + 1, tp.counters + 2, 1 << 24);
    DCHK(hipGetLastError());
  }
  int counters[3];
  DCHK(hipMemcpyAsync(counters, tp.counters, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
  DCHK(hipMemcpyAsync(&flags, tp.flags, sizeof(int), hipMemcpyDeviceToHost, s));
  DCHK(hipStreamSynchronize(s));
  if (flags & kFlagTimeout) {
    free_device_analysis(out);
    return kErrTimeout;
  }
  out.max_row_len = counters[0];
  out.nlev = counters[1] + 1;
  const int nlev = out.nlev;
  int lev_bits = 1;
  while (lev_bits < 31 && (1ll << lev_bits) < nlev) ++lev_bits;

  // stable radix sorts: positions by (level, length class); jlev by level
  DALLOC(tp.key, n);
  DALLOC(tp.key_s, n);
  DALLOC(tp.rows, n);
  DALLOC(tp.lkey, n);
  DALLOC(tp.lkey_s, n);
  DALLOC(tp.rows2, n);
  DALLOC(out.pos_row, n);
  DALLOC(out.jlev, n);
  k_keys<<<blocks(n), 256, 0, s>>>(n, out.level, out.depcnt, tp.key, tp.rows, tp.lkey, tp.rows2);
  DCHK(hipGetLastError());
  size_t b1 = 0, b2 = 0, b3 = 0;
  DCHK(rocprim::radix_sort_pairs(nullptr, b1, tp.key, tp.key_s, tp.rows, out.pos_row,
                                 static_cast<unsigned>(n), 0, 5 + lev_bits, s));
  DCHK(rocprim::radix_sort_pairs(nullptr, b2, tp.lkey, tp.lkey_s, tp.rows2, out.jlev,
                                 static_cast<unsigned>(n), 0, lev_bits, s));
  DALLOC(tp.cnt, static_cast<int64_t>(n) + 1);
  DALLOC(out.off_ptr, static_cast<int64_t>(n) + 1);
  DCHK(rocprim::exclusive_scan(nullptr, b3, tp.cnt, out.off_ptr, 0, static_cast<size_t>(n) + 1,
                               rocprim::plus<int>(), s));
  size_t tb = std::max(b1, std::max(b2, b3));
  if (hipMalloc(&tp.tmp, tb > 0 ? tb : 1) != hipSuccess) {
    free_device_analysis(out);
    return kErrOom;
  }
  DCHK(rocprim::radix_sort_pairs(tp.tmp, b1, tp.key, tp.key_s, tp.rows, out.pos_row,
                                 static_cast<unsigned>(n), 0, 5 + lev_bits, s));
  DCHK(rocprim::radix_sort_pairs(tp.tmp, b2, tp.lkey, tp.lkey_s, tp.rows2, out.jlev,
                                 static_cast<unsigned>(n), 0, lev_bits, s));

  // inverse permutation, row lengths, level pointers, CSR pointers
  DALLOC(tp.pos_of, n);
  DALLOC(tp.ilev, static_cast<int64_t>(nlev) + 1);
  k_positions<<<blocks(static_cast<int64_t>(n) + 1), 256, 0, s>>>(n, nlev, out.pos_row, out.level,
                                                                   out.depcnt, tp.pos_of, tp.cnt,
                                                                   tp.ilev);
  DCHK(hipGetLastError());
  DCHK(rocprim::exclusive_scan(tp.tmp, b3, tp.cnt, out.off_ptr, 0, static_cast<size_t>(n) + 1,
                               rocprim::plus<int>(), s));
  out.off_ptr_h.resize(static_cast<size_t>(n) + 1);
  out.ilev.resize(static_cast<size_t>(nlev) + 1);
  DCHK(hipMemcpyAsync(out.off_ptr_h.data(), out.off_ptr, (static_cast<size_t>(n) + 1) * sizeof(int),
                      hipMemcpyDeviceToHost, s));
  DCHK(hipMemcpyAsync(out.ilev.data(), tp.ilev, (static_cast<size_t>(nlev) + 1) * sizeof(int),
                      hipMemcpyDeviceToHost, s));
  DCHK(hipStreamSynchronize(s));
  out.noff = out.off_ptr_h[n];

  // the level-ordered copy of the off-diagonal pattern
  DALLOC(out.off_col, out.noff);
  DALLOC(out.off_pos, out.noff);
  DALLOC(out.off_src, out.noff);
  DALLOC(out.diag_src, n);
  k_offdiag<<<blocks(n), 256, 0, s>>>(n, unit_diag, row_ptr, col, out.pos_row, tp.pos_of,
                                       out.off_ptr, out.off_col, out.off_pos, out.off_src,
                                       out.diag_src);
  DCHK(hipGetLastError());
  DCHK(hipStreamSynchronize(s));
  return kOk;
}

}  // namespace sptrsv

namespace sptrsv {

int device_transpose(int n, int64_t nnz, const int* row_ptr, const int* col, hipStream_t s,
                     int** rpT, int** colT, int** srcT) {
  *rpT = *colT = *srcT = nullptr;
  if (n < 1 || nnz < 0 || nnz > INT32_MAX) return kErrNotSupported;
  int *keys = nullptr, *keys_s = nullptr, *vals = nullptr, *row_of = nullptr;
  void* tmp = nullptr;
  int st = kOk;
  auto cleanup = [&]() {
    for (void* p : {static_cast<void*>(keys), static_cast<void*>(keys_s), static_cast<void*>(vals),
                    static_cast<void*>(row_of), tmp})
      if (p) (void)hipFree(p);
  };
  if (dmalloc(&keys_s, nnz) || dmalloc(&vals, nnz) || dmalloc(&row_of, nnz) ||
      dmalloc(rpT, static_cast<int64_t>(n) + 1) || dmalloc(colT, nnz) || dmalloc(srcT, nnz)) {
    st = kErrOom;
  }
  int col_bits = 1;
  while (col_bits < 31 && (1ll << col_bits) < n) ++col_bits;
  if (!st && nnz > 0) {
    // entries by column, stably: (column, entry) ascending, i.e. the rows of
    // T^T with their columns (rows of T) strictly increasing
    if (dmalloc(&keys, nnz) ||
        hipMemcpyAsync(keys, col, static_cast<size_t>(nnz) * sizeof(int), hipMemcpyDeviceToDevice,
                       s) != hipSuccess) {
      st = kErrOom;
    } else {
      k_fill_iota<<<blocks(nnz), 256, 0, s>>>(vals, nnz);
      size_t tb = 0;
      if (rocprim::radix_sort_pairs(nullptr, tb, keys, keys_s, vals, *srcT,
                                    static_cast<unsigned>(nnz), 0, col_bits, s) != hipSuccess ||
          hipMalloc(&tmp, tb > 0 ? tb : 1) != hipSuccess ||
          rocprim::radix_sort_pairs(tmp, tb, keys, keys_s, vals, *srcT, static_cast<unsigned>(nnz),
                                    0, col_bits, s) != hipSuccess)
        st = kErrHip;
    }
  }
  if (!st) {
    k_row_of<<<blocks(n), 256, 0, s>>>(n, row_ptr, row_of);
    k_transpose_fill<<<blocks(nnz > 0 ? nnz : 1), 256, 0, s>>>(n, nnz, keys_s, *srcT, row_of, *colT,
                                                               *rpT);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) st = kErrHip;
  }
  cleanup();
  if (st) {
    for (int** p : {rpT, colT, srcT})
      if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
      }
  }
  return st;
}

int device_value_sources(int n, int64_t noff_f, const int* off_src_f, const int* diag_src_f,
                         int64_t nnz, const int* srcT, DeviceAnalysis& t, hipStream_t s) {
  int* loc = nullptr;
  if (dmalloc(&loc, nnz)) return kErrOom;
  const int64_t tot_f = noff_f > n ? noff_f : n;
  const int64_t tot_t = t.noff > n ? t.noff : n;
  k_value_loc<<<blocks(tot_f), 256, 0, s>>>(n, noff_f, off_src_f, diag_src_f, loc);
  k_compose_src<<<blocks(tot_t), 256, 0, s>>>(n, t.noff, srcT, loc, t.off_src, t.diag_src);
  int st = kOk;
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) st = kErrHip;
  (void)hipFree(loc);
  return st;
}

int device_concat(const std::vector<ConcatSystem>& systems, int vb, int* rp_cat, int* col_cat,
                  void* vals_cat, hipStream_t s) {
  const int count = static_cast<int>(systems.size());
  std::vector<SysDesc> host(count);
  int64_t roff = 0, eoff = 0, maxw = 1;
  for (int k = 0; k < count; ++k) {
    const ConcatSystem& c = systems[k];
    host[k] = SysDesc{c.row_ptr, c.col, c.vals, c.n, c.nnz, static_cast<int>(roff),
                      static_cast<int>(eoff)};
    roff += c.n;
    eoff += c.nnz;
    maxw = std::max<int64_t>(maxw, std::max<int64_t>(c.n, c.nnz));
  }
  SysDesc* dsys = nullptr;
  int* flags = nullptr;
  int st = kOk;
  if (dmalloc(&dsys, count) || dmalloc(&flags, 1)) st = kErrOom;
  int f = 0;
  if (!st && (hipMemcpyAsync(dsys, host.data(), count * sizeof(SysDesc), hipMemcpyHostToDevice, s) !=
                  hipSuccess ||
              hipMemsetAsync(flags, 0, sizeof(int), s) != hipSuccess))
    st = kErrHip;
  if (!st) {
    const int bx = static_cast<int>(std::min<int64_t>((maxw + 255) / 256, 1024));
    k_concat<<<dim3(bx, count), 256, 0, s>>>(dsys, vb, rp_cat, col_cat,
                                             static_cast<unsigned char*>(vals_cat), flags);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&f, flags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = kErrHip;
  }
  if (!st) {
    // the last row pointer: total nnz
    const int last = static_cast<int>(eoff);
    if (hipMemcpy(rp_cat + roff, &last, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) st = kErrHip;
  }
  if (dsys) (void)hipFree(dsys);
  if (flags) (void)hipFree(flags);
  if (!st && f) st = kErrNotSupported;
  return st;
}

}  // namespace sptrsv
