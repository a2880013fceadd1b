// C ABI of libsptrsv (include/sptrsv.h): handle lifetime, analysis upload,
// schedule selection and launch sequencing.  Section references are to Li,
// arXiv:1710.04985.
#include "sptrsv.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "analysis.hpp"
#include "analysis_gpu.hpp"
#include "api_internal.hpp"
#include "column.hpp"
#include "probe.hpp"
#include "kernels.hpp"

using namespace sptrsv;

namespace {

struct WaveLists {
  int* ptr = nullptr;
  int* list = nullptr;
};

struct ChunkEntry {
  DevChunks d;
  std::vector<int> level_chunk;   // host copy: chunk range of every level
  std::vector<int> h_start, h_meta;
  int max_lg = 0;
  // (wavefronts, regions, wavefronts per workgroup)
  std::map<std::tuple<int, int, int>, WaveLists> waves;
};

// Push lists of one plan (column-wise solves) and their chunk tables.
struct PushState {
  bool built = false;
  DevPush d;
  std::vector<int> h_ptr;
  std::map<std::pair<int, int>, ChunkEntry> chunks;   // (group, epl)
};

struct PlanState {
  bool built = false;
  HostPlan h;
  DevPlan d;
  // analysed on the device: the host plan holds only nlev, ilev, pos_ilev
  // and off_ptr until something needs the rest (ensure_plan_host), which is
  // then downloaded from d and the analysis arrays below
  bool host_complete = true;
  int* a_level = nullptr;
  int* a_depcnt = nullptr;
  int* a_jlev = nullptr;
  PushState push;
  void* vals_buf = nullptr;       // [noff + 2n] values: off-diagonals, diagonal, 1/diagonal
  // (group, epl, rows_fixed, rows_per_lane)
  std::map<std::tuple<int, int, int, int>, ChunkEntry> chunks;
  // column-batched tables of the one-RHS chunking: (group, epl, columns)
  std::map<std::tuple<int, int, int>, ChunkEntry> col_chunks;
};

// Workgroup of the resident block kernel (SPTRSV_OPT_BLOCK_RESIDENT): the
// copy in and out of LDS takes every thread, the level walk one wavefront.
constexpr int kResidentThreads = 1024;

// Block-ordered plan (SPTRSV_ALGO_BLOCK) of one direction, on the device.
struct BlockState {
  bool built = false;
  PlanState ps;
  BlockInfo info;
  int* seg_row0 = nullptr;
  int* seg_base = nullptr;
  int* lev_pos = nullptr;
  int64_t res_bytes = -1;   // LDS bytes of the resident kernel (-1: some system needs wider indices)
  ChunkEntry dummy;   // unused chunk table (the block kernel needs none)
};

struct Config {
  int algo;
  int group;
  int epl;
  int sync;
  int rpl;    // rows per lane
  int grid;   // persistent workgroups, 0 = default
  int assign; // sptrsv_assign
  int poll = 1;  // waits: 1 overlapped rounds over all slots, 0 single rounds of pending ones
  int stride = 1;  // static schedules, one right-hand side: elements between xp values
  int mrows = 0;   // static schedule, several right-hand sides: rows per lane group
                   // (1, 2, 4; 0 = by the number of right-hand sides)
};

std::mutex g_tune_mu;
std::map<uint64_t, Config> g_tune_cache;

// Where a solve keeps its position-ordered solution.  By default in the
// handle's own buffer (grown on demand); sptrsv_solve_noalloc passes a
// caller-side buffer of fixed capacity instead and forbids every allocation
// (work tables not built yet -> SPTRSV_ERR_NOT_SUPPORTED).
struct SolveExt {
  void* xp = nullptr;          // external buffer, or null for the handle's own
  int64_t xp_bytes = 0;        // its capacity
  bool no_alloc = false;
};

// Device buffer shared by a handle and the graphs captured with it: a buffer
// the handle replaces (a larger position-ordered solution) stays allocated
// until the last graph that baked its address into a kernel is destroyed.
struct DevBuffer {
  void* p = nullptr;
  DevBuffer() = default;
  DevBuffer(const DevBuffer&) = delete;
  DevBuffer& operator=(const DevBuffer&) = delete;
  ~DevBuffer() {
    if (p) (void)hipFree(p);   // hipFree waits for the device before freeing
  }
};

}  // namespace

struct sptrsv_handle_s {
  int n = 0;
  int64_t nnz = 0;
  sptrsv_dtype dtype = SPTRSV_F64;
  bool upper = false;
  bool unit = false;
  size_t vb = 8;
  int device = 0;
  int num_cu = 256;
  int lds_limit = 65536;          // bytes of LDS one workgroup may use
  int block_resident = 1;         // block schedule: whole system in LDS when it fits
  int coop = 0;                   // persistent static grids: cooperative launch
  std::vector<int> rp_h, col_h;   // caller's pattern (host copy)
  PlanState fwd, trn;
  // device setup: the handle's own device copy of the pattern (for T^T and
  // batched handles the concatenated pattern), downloaded to rp_h / col_h
  // only when the host needs it
  bool pattern_host = true;
  int* rp_dev = nullptr;
  int* col_dev = nullptr;
  void* col_acc = nullptr;         // column-wise solves: accumulators [n]
  int* col_cnt = nullptr;          // and arrival counts [n]
  int setup = SPTRSV_SETUP_HOST;  // route the analysis took
  double setup_ms = 0.0;           // wall time of the analysis call
  BlockState blk[2];               // block-ordered plans of T and T^T
  DevScratch scratch;
  std::shared_ptr<DevBuffer> xp_buf;   // position-ordered solution(s) of the solve kernels
  void* xp = nullptr;             // xp_buf->p
  int64_t xp_elems = 0;
  int live_graphs = 0;            // graphs captured from this handle, not yet destroyed
  void* bp = nullptr;             // several right-hand sides in position order
  int64_t bp_elems = 0;
  // batched handles keep the concatenated pattern and values on the device
  bool batched = false;
  std::vector<int> sys_n, sys_nnz;
  int* rp_cat = nullptr;
  int* col_cat = nullptr;
  void* vals_cat = nullptr;
  // options
  int algo = SPTRSV_ALGO_AUTO;
  int group = 0;
  int epl = 4;
  int sync = SPTRSV_SYNC_VALUE;
  int spin_limit = 1 << 22;
  int grid = 0;
  int timing = 0;
  int wg = 64;
  int rpl = 1;
  int assign = SPTRSV_ASSIGN_STATIC;
  int poll = 1;
  int xp_stride = 1;
  int mrows = 0;
  int res_limit = 1 << 20;
  // schedule options the caller set (the defaults of the others follow the
  // pattern, see resolve)
  unsigned set_mask = 0;
  int max_level = -1;   // rows of the widest level of the forward plan (-1: not computed)
  // autotuner result
  bool tuned = false;
  Config tuned_cfg{SPTRSV_ALGO_SELF, 0, 4, SPTRSV_SYNC_VALUE, 1, 0, SPTRSV_ASSIGN_STATIC};
  std::map<int, Config> tuned_multi;   // sptrsv_tune_multi's choice per nrhs
  uint64_t hash = 0;               // pattern hash, computed by the first sptrsv_tune
  bool hash_valid = false;
  // timing
  std::map<std::pair<int, int>, int> occupancy;   // (kernel kind, wg) -> blocks per CU
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  size_t ev_used = 0;
  double acc_ms = 0.0;
  int64_t acc_count = 0;
  hipStream_t last_stream = nullptr;
  // cross-stream ordering of the work that uses the handle's buffers
  hipEvent_t order_ev = nullptr;
  hipStream_t order_stream = nullptr;
  bool order_pending = false;
};

struct sptrsv_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  sptrsv_handle_t owner = nullptr;
  std::shared_ptr<DevBuffer> xp_keep;   // the position-ordered buffer the graph's kernels use
};

#define HIPCHK(expr)                          \
  do {                                        \
    if ((expr) != hipSuccess) return kErrHip; \
  } while (0)

namespace {

template <typename T> T* dalloc(size_t count, int* err) {
  if (count == 0) count = 1;
  void* p = nullptr;
  if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
    *err = kErrOom;
    return nullptr;
  }
  return static_cast<T*>(p);
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

void free_entry(ChunkEntry& e) {
  dfree(e.d.start);
  dfree(e.d.meta);
  dfree(e.d.col);
  for (auto& w : e.waves) {
    dfree(w.second.ptr);
    dfree(w.second.list);
  }
}

void free_chunks(PlanState& ps) {
  for (auto& kv : ps.chunks) free_entry(kv.second);
  ps.chunks.clear();
  for (auto& kv : ps.col_chunks) free_entry(kv.second);
  ps.col_chunks.clear();
  for (auto& kv : ps.push.chunks) free_entry(kv.second);
  ps.push.chunks.clear();
}

// Per-wavefront chunk lists of a static schedule over W wavefronts (built on
// first use and kept; synchronous upload).
const WaveLists* get_wave_lists(ChunkEntry& ch, int W, int regions, int wpb, int* err,
                                bool no_alloc = false) {
  const auto key = std::make_tuple(W, regions, wpb);
  auto it = ch.waves.find(key);
  if (it != ch.waves.end()) return &it->second;
  if (no_alloc) {
    *err = kErrNotSupported;
    return nullptr;
  }
  ChunkTable t;
  t.start = ch.h_start;
  t.meta = ch.h_meta;
  t.level_chunk = ch.level_chunk;
  std::vector<int> ptr, list;
  build_wave_lists(t, W, regions, ptr, list, wpb);
  WaveLists wl;
  int st = kOk;
  wl.ptr = dalloc<int>(ptr.size(), &st);
  wl.list = dalloc<int>(list.size(), &st);
  if (st || hipMemcpy(wl.ptr, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      (!list.empty() &&
       hipMemcpy(wl.list, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)) {
    dfree(wl.ptr);
    dfree(wl.list);
    *err = st ? st : kErrHip;
    return nullptr;
  }
  return &(ch.waves[key] = wl);
}

void free_push(PushState& p) {
  for (auto& kv : p.chunks) free_entry(kv.second);
  dfree(p.d.ptr);
  dfree(p.d.dst);
  dfree(p.d.src);
  dfree(p.d.val);
  p = PushState();
}

void free_plan(PlanState& ps) {
  free_chunks(ps);
  dfree(ps.d.off_ptr);
  dfree(ps.d.off_col);
  dfree(ps.d.off_pos);
  dfree(ps.d.off_src);
  dfree(ps.d.diag_src);
  dfree(ps.d.pos_row);
  dfree(ps.d.row_pos);
  dfree(ps.vals_buf);
  dfree(ps.a_level);
  dfree(ps.a_depcnt);
  dfree(ps.a_jlev);
  free_push(ps.push);
  ps.d = DevPlan();
  ps.vals_buf = nullptr;
  ps.a_level = ps.a_depcnt = ps.a_jlev = nullptr;
  ps.host_complete = true;
  ps.built = false;
}

int upload_ints(int** dst, const std::vector<int>& v, hipStream_t s) {
  int err = kOk;
  *dst = dalloc<int>(v.size(), &err);
  if (!*dst) return err;
  if (!v.empty())
    HIPCHK(hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, s));
  return kOk;
}

// Uploads the host plan; values are gathered separately.
int upload_plan(PlanState& ps, size_t vb, hipStream_t s) {
  const HostPlan& h = ps.h;
  DevPlan& d = ps.d;
  d.n = h.n;
  d.nlev = h.nlev;
  d.noff = h.noff;
  int st;
  if ((st = upload_ints(&d.off_ptr, h.off_ptr, s))) return st;
  if ((st = upload_ints(&d.off_col, h.off_col, s))) return st;
  if ((st = upload_ints(&d.off_pos, h.off_pos, s))) return st;
  if ((st = upload_ints(&d.off_src, h.off_src, s))) return st;
  if ((st = upload_ints(&d.diag_src, h.diag_src, s))) return st;
  if ((st = upload_ints(&d.pos_row, h.pos_row, s))) return st;
  int err = kOk;
  ps.vals_buf = dalloc<char>((static_cast<size_t>(h.noff) + 2 * static_cast<size_t>(h.n)) * vb, &err);
  if (!ps.vals_buf) return err;
  d.off_val = ps.vals_buf;
  d.diag = static_cast<char*>(ps.vals_buf) + static_cast<size_t>(h.noff) * vb;
  d.dinv = static_cast<char*>(d.diag) + static_cast<size_t>(h.n) * vb;
  ps.built = true;
  return kOk;
}

// Completes the host plan of a plan analysed on the device: every plan
// array is downloaded once (blocking).
int ensure_plan_host(PlanState& ps) {
  if (ps.host_complete) return kOk;
  const size_t n = static_cast<size_t>(ps.h.n);
  HostPlan& p = ps.h;
  const DevPlan& d = ps.d;
  p.level.resize(n);
  p.depcnt.resize(n);
  p.jlev.resize(n);
  p.pos_row.resize(n);
  p.off_col.resize(p.noff);
  p.off_pos.resize(p.noff);
  p.off_src.resize(p.noff);
  p.diag_src.resize(n);
  const std::pair<int*, const int*> parts[] = {
      {p.level.data(), ps.a_level},  {p.depcnt.data(), ps.a_depcnt},
      {p.jlev.data(), ps.a_jlev},    {p.pos_row.data(), d.pos_row},
      {p.off_col.data(), d.off_col}, {p.off_pos.data(), d.off_pos},
      {p.off_src.data(), d.off_src}, {p.diag_src.data(), d.diag_src}};
  const size_t counts[] = {n, n, n, n, static_cast<size_t>(p.noff), static_cast<size_t>(p.noff),
                           static_cast<size_t>(p.noff), n};
  for (size_t q = 0; q < sizeof(counts) / sizeof(counts[0]); ++q)
    if (counts[q] > 0)
      HIPCHK(hipMemcpy(parts[q].first, parts[q].second, counts[q] * sizeof(int),
                       hipMemcpyDeviceToHost));
  ps.host_complete = true;
  return kOk;
}

// The handle's pattern on the host (downloaded once from its device copy).
int ensure_pattern_host(sptrsv_handle_t h) {
  if (h->pattern_host) return kOk;
  h->rp_h.resize(static_cast<size_t>(h->n) + 1);
  h->col_h.resize(h->nnz);
  HIPCHK(hipMemcpy(h->rp_h.data(), h->rp_dev, (static_cast<size_t>(h->n) + 1) * sizeof(int),
                   hipMemcpyDeviceToHost));
  if (h->nnz > 0)
    HIPCHK(hipMemcpy(h->col_h.data(), h->col_dev, static_cast<size_t>(h->nnz) * sizeof(int),
                     hipMemcpyDeviceToHost));
  h->pattern_host = true;
  return kOk;
}

// Pattern and forward plan on the host.
int ensure_host_plan(sptrsv_handle_t h) {
  if (const int st = ensure_pattern_host(h)) return st;
  return ensure_plan_host(h->fwd);
}

int gather(sptrsv_handle_t h, PlanState& ps, const void* vals, hipStream_t s) {
  hipError_t e;
  if (h->dtype == SPTRSV_F64)
    e = launch_gather<double>(ps.d, static_cast<const double*>(vals), h->scratch.status, s);
  else
    e = launch_gather<float>(ps.d, static_cast<const float*>(vals), h->scratch.status, s);
  return e == hipSuccess ? kOk : kErrHip;
}

int read_status(sptrsv_handle_t h, hipStream_t s, bool clear) {
  int st = 0;
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemcpy(&st, h->scratch.status, sizeof(int), hipMemcpyDeviceToHost));
  if (clear && st) {
    const int zero = 0;
    HIPCHK(hipMemcpy(h->scratch.status, &zero, sizeof(int), hipMemcpyHostToDevice));
  }
  if (st & kStatusNotResident) return kErrNotResident;
  if (st & kStatusTimeout) return kErrTimeout;
  if (st & kStatusZeroPivot) return kErrZeroPivot;
  return kOk;
}

int install_device_plan(sptrsv_handle_t h, PlanState& ps, DeviceAnalysis& da, bool upper);

// Builds the analysis of T^T: rows of T^T are the columns of T; each value is
// taken from the forward plan's value buffer (so the caller's vals need not
// outlive the analysis).  A handle analysed on the device builds it on the
// device too (transposed pattern by a stable radix sort, the device level
// sweep on it, value sources composed there); otherwise on the host.
int build_transpose(sptrsv_handle_t h, hipStream_t s) {
  if (h->trn.built) return kOk;
  const int n = h->n;
  if (h->rp_dev && n > 0) {
    int *rT = nullptr, *cT = nullptr, *sT = nullptr;
    int st = device_transpose(n, h->nnz, h->rp_dev, h->col_dev, s, &rT, &cT, &sT);
    DeviceAnalysis da;
    if (!st) st = device_analysis(n, h->nnz, rT, cT, !h->upper, h->unit, h->num_cu, s, da);
    if (!st)
      st = device_value_sources(n, h->fwd.d.noff, h->fwd.d.off_src, h->fwd.d.diag_src, h->nnz, sT,
                                da, s);
    for (int* q : {rT, cT, sT}) dfree(q);
    if (!st) st = install_device_plan(h, h->trn, da, !h->upper);
    if (!st) st = gather(h, h->trn, h->fwd.vals_buf, s);
    if (!st && hipStreamSynchronize(s) != hipSuccess) st = kErrHip;
    if (st) {
      free_device_analysis(da);
      free_plan(h->trn);
    }
    if (st != kErrNotSupported) return st;   // else the host route below decides
  }
  if (const int st = ensure_host_plan(h)) return st;
  const HostPlan& f = h->fwd.h;
  // location of every caller entry in the forward value buffer
  std::vector<int> loc(h->nnz, -1);
  for (int k = 0; k < n; ++k) {
    for (int o = f.off_ptr[k]; o < f.off_ptr[k + 1]; ++o) loc[f.off_src[o]] = o;
    if (f.diag_src[k] >= 0) loc[f.diag_src[k]] = static_cast<int>(f.noff) + k;
  }
  std::vector<int> rT, cT, sT;
  transpose_pattern(n, h->rp_h.data(), h->col_h.data(), rT, cT, sT);
  for (auto& v : sT) v = loc[v];
  build_plan(n, rT.data(), cT.data(), sT.data(), !h->upper, h->unit, h->trn.h);
  int st = upload_plan(h->trn, h->vb, s);
  if (!st) st = gather(h, h->trn, h->fwd.vals_buf, s);
  if (!st && hipStreamSynchronize(s) != hipSuccess) st = kErrHip;
  if (st) free_plan(h->trn);   // a later call starts over instead of using half a plan
  return st;
}

void free_block(BlockState& b);

// Builds the block-ordered plan of direction `dir` (0: T, 1: T^T): one
// segment per system of a batched handle, else one; values are gathered from
// the direction's level-ordered plan.  Blocking (uploads synchronously).
int build_block(sptrsv_handle_t h, int dir, hipStream_t s) {
  BlockState& b = h->blk[dir];
  if (b.built) return kOk;
  PlanState& base = dir ? h->trn : h->fwd;
  if (const int st = ensure_plan_host(base)) return st;
  std::vector<int> seg_row0(1, 0);
  if (h->batched)
    for (int ni : h->sys_n) seg_row0.push_back(seg_row0.back() + ni);
  else
    seg_row0.push_back(h->n);
  build_block_plan(base.h, seg_row0, b.ps.h, b.info);
  b.res_bytes = block_resident_bytes(b.ps.h, b.info, h->vb);
  int st = upload_plan(b.ps, h->vb, s);
  if (!st) st = upload_ints(&b.seg_row0, b.info.seg_row0, s);
  if (!st) st = upload_ints(&b.seg_base, b.info.seg_base, s);
  if (!st) st = upload_ints(&b.lev_pos, b.info.lev_pos, s);
  if (!st) st = gather(h, b.ps, base.vals_buf, s);
  if (!st && hipStreamSynchronize(s) != hipSuccess) st = kErrHip;
  if (st) {
    free_block(b);   // nothing half-built stays behind
    return st;
  }
  b.built = true;
  return kOk;
}

// Uploads chunk table t into a new entry (synchronous copies: the table may
// be built the first time a solve is issued, and t dies with the caller).
bool upload_chunks(const ChunkTable& t, ChunkEntry& e, int* err);

ChunkEntry* get_chunks(sptrsv_handle_t h, PlanState& ps, int group, int epl, int rows_fixed,
                       int rpl, int* err, bool no_alloc = false) {
  (void)h;
  auto key = std::make_tuple(group, epl, rows_fixed, rpl);
  auto it = ps.chunks.find(key);
  if (it != ps.chunks.end()) return &it->second;
  if (no_alloc) {
    *err = kErrNotSupported;
    return nullptr;
  }
  ChunkTable t;
  build_chunks(ps.h, group, epl, rows_fixed, rpl, t);
  ChunkEntry e;
  if (!upload_chunks(t, e, err)) return nullptr;
  return &(ps.chunks[key] = e);
}

// Chunks over the push lists of a plan: rows of one level get lanes by the
// length of their push list.
ChunkEntry* get_push_chunks(PlanState& ps, int group, int epl, int* err, bool no_alloc = false) {
  auto key = std::make_pair(group, epl);
  auto it = ps.push.chunks.find(key);
  if (it != ps.push.chunks.end()) return &it->second;
  if (no_alloc) {
    *err = kErrNotSupported;
    return nullptr;
  }
  HostPlan view;
  view.n = ps.h.n;
  view.nlev = ps.h.nlev;
  view.pos_ilev = ps.h.pos_ilev;
  view.off_ptr = ps.push.h_ptr;
  ChunkTable t;
  build_chunks(view, group, epl, 0, 1, t);
  ChunkEntry e;
  if (!upload_chunks(t, e, err)) return nullptr;
  return &(ps.push.chunks[key] = e);
}

bool upload_chunks(const ChunkTable& t, ChunkEntry& e, int* err) {
  e.level_chunk = t.level_chunk;
  e.h_start = t.start;
  e.h_meta = t.meta;
  e.max_lg = t.max_lg;
  e.d.count = static_cast<int>(t.start.size());
  int st;
  e.d.start = dalloc<int>(t.start.size(), &st);
  e.d.meta = dalloc<int>(t.meta.size(), &st);
  if (!e.d.start || !e.d.meta) {
    dfree(e.d.start);
    dfree(e.d.meta);
    *err = kErrOom;
    return false;
  }
  if (!t.start.empty() &&
      (hipMemcpy(e.d.start, t.start.data(), t.start.size() * sizeof(int), hipMemcpyHostToDevice) !=
           hipSuccess ||
       hipMemcpy(e.d.meta, t.meta.data(), t.meta.size() * sizeof(int), hipMemcpyHostToDevice) !=
           hipSuccess)) {
    dfree(e.d.start);
    dfree(e.d.meta);
    *err = kErrHip;
    return false;
  }
  return true;
}

// Column-batched chunk table for `ncols` right-hand sides solved at once by
// the one-RHS static kernel: every level lists the chunks of `base` once per
// column (column-major inside the level), each tagged with its column, so a
// wavefront's list stays in level order and every column is chunked exactly
// as its own one-RHS solve.  Built on first use and kept.
ChunkEntry* get_col_chunks(PlanState& ps, int group, int epl, int ncols, const ChunkEntry& base,
                           int* err) {
  const auto key = std::make_tuple(group, epl, ncols);
  auto it = ps.col_chunks.find(key);
  if (it != ps.col_chunks.end()) return &it->second;
  const int nlev = static_cast<int>(base.level_chunk.size()) - 1;
  const int64_t total = static_cast<int64_t>(base.h_start.size()) * ncols;
  if (total > INT32_MAX) {
    *err = kErrTooLarge;
    return nullptr;
  }
  ChunkEntry e;
  e.max_lg = base.max_lg;
  e.level_chunk.assign(nlev + 1, 0);
  e.h_start.reserve(total);
  e.h_meta.reserve(total);
  std::vector<int> col;
  col.reserve(total);
  for (int m = 0; m < nlev; ++m) {
    e.level_chunk[m] = static_cast<int>(e.h_start.size());
    for (int q = 0; q < ncols; ++q)
      for (int c = base.level_chunk[m]; c < base.level_chunk[m + 1]; ++c) {
        e.h_start.push_back(base.h_start[c]);
        e.h_meta.push_back(base.h_meta[c]);
        col.push_back(q);
      }
  }
  if (nlev >= 0) e.level_chunk[nlev] = static_cast<int>(e.h_start.size());
  e.d.count = static_cast<int>(total);
  int st = kOk;
  e.d.start = dalloc<int>(e.h_start.size(), &st);
  e.d.meta = dalloc<int>(e.h_meta.size(), &st);
  e.d.col = dalloc<int>(col.size(), &st);
  const size_t bytes = e.h_start.size() * sizeof(int);
  if (st || !e.d.start || !e.d.meta || !e.d.col ||
      (bytes && (hipMemcpy(e.d.start, e.h_start.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
                 hipMemcpy(e.d.meta, e.h_meta.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
                 hipMemcpy(e.d.col, col.data(), bytes, hipMemcpyHostToDevice) != hipSuccess))) {
    free_entry(e);
    *err = st ? st : kErrHip;
    return nullptr;
  }
  return &(ps.col_chunks[key] = e);
}

// Option bits of set_mask: options set explicitly, which the pattern-based
// defaults of resolve() leave alone.
constexpr unsigned kSetGrid = 1, kSetAssign = 2, kSetStride = 4;

// Rows of the widest level of the forward plan (cached: the pattern of a
// handle never changes).
int widest_level(sptrsv_handle_t h) {
  if (h->max_level < 0) {
    const std::vector<int>& il = h->fwd.h.pos_ilev;
    int w = 0;
    for (size_t m = 0; m + 1 < il.size(); ++m) w = std::max(w, il[m + 1] - il[m]);
    h->max_level = w;
  }
  return h->max_level;
}

// The schedule a solve uses: the autotuner's choice if there is one, else the
// options.  Options left at their defaults follow features of the pattern
// (deterministic, no trials, and no choice below changes the result bits:
// every one keeps the lane rule).  The thresholds are where the autotuner's
// picks changed on the measured workloads:
//  * one system, one lane per row, at most 64 rows per level, small enough
//    for the whole system to sit in LDS: the block schedule (it runs without
//    any global synchronisation; 2-D 64x64: 0.054 ms against 0.095);
//  * otherwise self-scheduled; levels of at most 4,096 rows on average take
//    the ticket schedule (ILU(0) 96^3, the 2-D 64x64 triangle) unless rows
//    exceed 64 entries; the others the XCD-regional static one;
//  * rows longer than 64 entries, or levels of more than 8,192 rows on
//    average, take two wavefronts per CU (power-law, batched ILU(0));
//  * rows longer than 64 entries take 32-byte slots for the solution
//    (power-law: 0.72 against 0.82 ms packed).
Config resolve(sptrsv_handle_t h) {
  if (h->tuned) return h->tuned_cfg;
  Config c{h->algo, h->group, h->epl, h->sync, h->rpl, h->grid, h->assign};
  c.poll = h->poll;
  c.stride = h->xp_stride;
  c.mrows = h->mrows;
  const HostPlan& p = h->fwd.h;
  const int64_t n = h->n, nlev = p.nlev > 0 ? p.nlev : 1;
  if (c.algo == SPTRSV_ALGO_AUTO) {
    const bool one_lane = h->group == 1 || (h->group == 0 && p.max_row_len <= h->epl);
    const int64_t lds = static_cast<int64_t>(h->vb) * (2 * n + p.noff + 2) + 2 * (n + 1) +
                        2 * (p.noff + 1) + 2 * (nlev + 1);
    if (!h->batched && one_lane && h->block_resident && n <= 65535 && p.noff <= 65535 &&
        lds <= h->lds_limit && widest_level(h) <= 64) {
      c.algo = SPTRSV_ALGO_BLOCK;
      return c;
    }
    c.algo = SPTRSV_ALGO_SELF;
  }
  if (c.algo != SPTRSV_ALGO_SELF || c.sync != SPTRSV_SYNC_VALUE) return c;
  const bool long_rows = p.max_row_len > 64;
  // (a slot width set explicitly asks for a static schedule: only those use it)
  if (!(h->set_mask & kSetAssign))
    c.assign = n <= 4096 * nlev && !long_rows && !(h->set_mask & kSetStride)
                   ? SPTRSV_ASSIGN_TICKET
                   : SPTRSV_ASSIGN_XCD;
  if (!(h->set_mask & kSetGrid) && (long_rows || n > 8192 * nlev)) c.grid = 2 * h->num_cu;
  if (!(h->set_mask & kSetStride) && long_rows) c.stride = 32 / h->vb;
  return c;
}

// Schedule of a solve with nrhs > 1 right-hand sides: sptrsv_tune_multi's
// choice for this nrhs if there is one, else the single-RHS schedule with a
// grid sized for several columns unless the grid option is set (each chunk
// then holds 64/nrhs rows, so a level has many more chunks to spread).
Config resolve_multi(sptrsv_handle_t h, int nrhs) {
  auto it = h->tuned_multi.find(nrhs);
  if (it != h->tuned_multi.end()) return it->second;
  Config c = resolve(h);
  // the block schedule solves one right-hand side; a default choice of it
  // becomes the self-scheduled solve here
  if (h->algo == SPTRSV_ALGO_AUTO && !h->tuned && c.algo == SPTRSV_ALGO_BLOCK)
    c.algo = SPTRSV_ALGO_SELF;
  // options left unset, by the column count (where sptrsv_tune_multi's picks
  // changed on 128^3 and ILU(0) 96^3): 2, 4, 8 wavefronts per CU from 2, 8,
  // 16 columns; XCD-regional lists up to 4 columns, round-robin beyond
  if (!(h->set_mask & kSetGrid))
    c.grid = (nrhs >= 16 ? 8 : nrhs >= 8 ? 4 : 2) * h->num_cu;
  if (!(h->set_mask & kSetAssign) && c.algo == SPTRSV_ALGO_SELF)
    c.assign = nrhs <= 4 ? SPTRSV_ASSIGN_XCD : SPTRSV_ASSIGN_STATIC;
  return c;
}

// Several right-hand sides on a pattern with rows longer than 64 entries
// and a lane rule that gives such rows several lanes: the multi-RHS kernels
// walk a row with one lane per column, so a long row costs one lane its
// whole length per column; solving the columns one after another with the
// single-RHS schedule is faster there (power-law, 16 columns: 36 ms at the
// best multi-RHS schedule, 16 x 0.72 ms this way).
bool multi_by_columns(const PlanState& ps, const Config& c) {
  return c.group != 1 && ps.h.max_row_len > 64 &&
         (c.algo == SPTRSV_ALGO_SELF || c.algo == SPTRSV_ALGO_LEVEL ||
          c.algo == SPTRSV_ALGO_BLOCK);
}

uint64_t tune_key(sptrsv_handle_t h) {
  return h->hash ^ (h->dtype == SPTRSV_F32 ? 0x9e3779b97f4a7c15ull : 0) ^
         (static_cast<uint64_t>(h->algo) << 56) ^ (static_cast<uint64_t>(h->group) << 48) ^
         (static_cast<uint64_t>(h->epl) << 32);
}

// Grows the position-ordered solution buffer to `elems` values.  Work the
// handle issued earlier may still use the old buffer: it is waited for
// through the handle's ordering event (not the whole device), and a graph
// captured with the old buffer keeps it alive (see DevBuffer).
int ensure_xp(sptrsv_handle_t h, int64_t elems) {
  if (h->xp_elems >= elems) return kOk;
  if (h->xp_buf && h->order_ev && h->order_pending) HIPCHK(hipEventSynchronize(h->order_ev));
  auto nb = std::make_shared<DevBuffer>();
  if (hipMalloc(&nb->p, static_cast<size_t>(elems > 0 ? elems : 1) * h->vb) != hipSuccess)
    return kErrOom;
  h->xp_buf = std::move(nb);   // frees the old buffer unless a graph holds it
  h->xp = h->xp_buf->p;
  h->xp_elems = elems;
  return kOk;
}

// Several right-hand sides: the position-ordered copy of B (grown like the
// solution buffer) and the plan's inverse permutation (built once).
int ensure_multi(sptrsv_handle_t h, PlanState& ps, int64_t elems, hipStream_t s) {
  if (h->bp_elems < elems) {
    if (h->bp && h->order_ev && h->order_pending) HIPCHK(hipEventSynchronize(h->order_ev));
    dfree(h->bp);
    h->bp = nullptr;
    h->bp_elems = 0;
    if (hipMalloc(&h->bp, static_cast<size_t>(elems > 0 ? elems : 1) * h->vb) != hipSuccess)
      return kErrOom;
    h->bp_elems = elems;
  }
  if (!ps.d.row_pos) {
    int err = kOk;
    ps.d.row_pos = dalloc<int>(static_cast<size_t>(h->n), &err);
    if (!ps.d.row_pos) return err;
    HIPCHK(launch_row_pos(h->n, ps.d.pos_row, ps.d.row_pos, s));
  }
  return kOk;
}

// Resident workgroups per CU of persistent kernel `kind` (0 value sync, 1 flag
// sync, 3 static value sync, 4 column-wise, 5 + log2(rows per lane group):
// static value sync with several right-hand sides); queried once per (kind,
// wg) and cached, so that solves under graph capture make no occupancy query.
int blocks_per_cu(sptrsv_handle_t h, int kind) {
  const auto key = std::make_pair(kind, h->wg);
  auto it = h->occupancy.find(key);
  if (it != h->occupancy.end()) return it->second;
  int per_cu;
  const bool dbl = h->dtype == SPTRSV_F64;
  if (kind == 0) per_cu = dbl ? self_value_blocks_per_cu<double>(h->wg) : self_value_blocks_per_cu<float>(h->wg);
  else if (kind == 1) per_cu = dbl ? self_flag_blocks_per_cu<double>(h->wg) : self_flag_blocks_per_cu<float>(h->wg);
  else if (kind == 3) per_cu = dbl ? self_static_blocks_per_cu<double>(h->wg) : self_static_blocks_per_cu<float>(h->wg);
  else if (kind >= 5) per_cu = dbl ? self_multi_blocks_per_cu<double>(h->wg, 1 << (kind - 5)) : self_multi_blocks_per_cu<float>(h->wg, 1 << (kind - 5));
  else per_cu = dbl ? column_self_blocks_per_cu<double>(h->wg) : column_self_blocks_per_cu<float>(h->wg);
  h->occupancy[key] = per_cu;
  return per_cu;
}

// Workgroups of a persistent launch: the explicit choice, else one
// wavefront per CU; never more than chunks need, than half of what the
// occupancy figure allows, or than 8 wavefronts per CU (a quarter of a CU's
// wave slots), so the all-resident schedules keep at least a factor of two
// below the reported capacity (their wavefronts also check residency when
// they start, whether the launch is cooperative or not).
int persistent_grid(sptrsv_handle_t h, int kind, int grid, int nchunks) {
  const int per_cu = blocks_per_cu(h, kind);
  const int waves_per_block = h->wg / 64;
  const int need = (nchunks + waves_per_block - 1) / waves_per_block;
  int g = grid > 0 ? grid : (h->num_cu + waves_per_block - 1) / waves_per_block;
  const int cap_per_cu = std::max(1, std::min(per_cu / 2, 8 / waves_per_block));
  g = std::min(g, cap_per_cu * h->num_cu);
  return std::max(1, std::min(g, need));
}

// Adds the recorded kernel times to the handle's totals and frees the event
// pairs for reuse (waits for the recorded stops).
int fold_timing(sptrsv_handle_t h) {
  for (size_t i = 0; i < h->ev_used; ++i) {
    HIPCHK(hipEventSynchronize(h->ev_pool[i].second));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, h->ev_pool[i].first, h->ev_pool[i].second));
    h->acc_ms += t;
    h->acc_count++;
  }
  h->ev_used = 0;
  return kOk;
}

constexpr size_t kMaxTimedSolves = 1024;   // event pairs kept before they are folded

void timing_begin(sptrsv_handle_t h, hipStream_t s, hipEvent_t* stop, bool no_alloc = false) {
  *stop = nullptr;
  if (!h->timing || no_alloc) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  if (h->ev_used == kMaxTimedSolves && fold_timing(h) != kOk) return;
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return;
    }
    h->ev_pool.emplace_back(a, b);
  }
  auto& pr = h->ev_pool[h->ev_used++];
  (void)hipEventRecord(pr.first, s);
  *stop = pr.second;
}

void timing_end(hipStream_t s, hipEvent_t stop) {
  if (stop) (void)hipEventRecord(stop, s);
}

// Occupancy kind of the static schedule: 3 with one right-hand side (mrows
// 0), 5, 6, 7 for the multi-RHS kernel with 1, 2, 4 rows per lane group.
int multi_kind(int mrows) { return mrows <= 0 ? 3 : mrows >= 4 ? 7 : mrows == 2 ? 6 : 5; }

// Wave-list key of the static schedule: (wavefronts, regions, wavefronts per
// workgroup).
std::tuple<int, int, int> static_key(sptrsv_handle_t h, const ChunkEntry& ch, const Config& c,
                                     int mrows = 0) {
  const int grid = persistent_grid(h, multi_kind(mrows), c.grid, ch.d.count);
  const int W = grid * (h->wg / 64);
  const int wpb = h->wg / 64;
  const int regions = (c.assign == SPTRSV_ASSIGN_XCD && W % (8 * wpb) == 0) ? 8 : 1;
  return std::make_tuple(W, regions, wpb);
}

bool static_lists_ready(sptrsv_handle_t h, const ChunkEntry& ch, const Config& c,
                        int mrows = 0) {
  return ch.waves.count(static_key(h, ch, c, mrows)) != 0;
}

const WaveLists* static_lists(sptrsv_handle_t h, ChunkEntry& ch, const Config& c, int* err,
                              int mrows = 0) {
  const auto key = static_key(h, ch, c, mrows);
  return get_wave_lists(ch, std::get<0>(key), std::get<1>(key), std::get<2>(key), err);
}

bool is_column(int algo) {
  return algo == SPTRSV_ALGO_COLUMN_LEVEL || algo == SPTRSV_ALGO_COLUMN_SELF;
}

// Push lists of plan ps, their values, and the column solves' scratch
// (blocking; built on first use).
int build_push_state(sptrsv_handle_t h, PlanState& ps, hipStream_t s) {
  if (ps.push.built) return kOk;
  if (const int st = ensure_plan_host(ps)) return st;
  std::vector<int> dst, src;
  build_push(ps.h, ps.push.h_ptr, dst, src);
  DevPush& d = ps.push.d;
  d.nnz = static_cast<int64_t>(dst.size());
  int err = kOk;
  d.ptr = dalloc<int>(ps.push.h_ptr.size(), &err);
  d.dst = dalloc<int>(dst.size(), &err);
  d.src = dalloc<int>(src.size(), &err);
  d.val = dalloc<char>(dst.size() * h->vb, &err);
  if (!h->col_acc) h->col_acc = dalloc<char>(static_cast<size_t>(h->n) * h->vb, &err);
  if (!h->col_cnt) h->col_cnt = dalloc<int>(static_cast<size_t>(h->n), &err);
  if (!err &&
      (hipMemcpy(d.ptr, ps.push.h_ptr.data(), ps.push.h_ptr.size() * sizeof(int),
                 hipMemcpyHostToDevice) != hipSuccess ||
       (!dst.empty() &&
        (hipMemcpy(d.dst, dst.data(), dst.size() * sizeof(int), hipMemcpyHostToDevice) !=
             hipSuccess ||
         hipMemcpy(d.src, src.data(), src.size() * sizeof(int), hipMemcpyHostToDevice) !=
             hipSuccess)) ||
       (h->dtype == SPTRSV_F64 ? launch_push_gather<double>(ps.d, d, s)
                               : launch_push_gather<float>(ps.d, d, s)) != hipSuccess ||
       hipStreamSynchronize(s) != hipSuccess))
    err = kErrHip;
  if (err) {
    free_push(ps.push);   // a later call starts over
    return err;
  }
  ps.push.built = true;
  return kOk;
}

// Re-gathers the push values of every built plan after a value update.
int regather_push(sptrsv_handle_t h, hipStream_t s) {
  for (PlanState* ps : {&h->fwd, &h->trn}) {
    if (!ps->push.built) continue;
    const hipError_t e = h->dtype == SPTRSV_F64 ? launch_push_gather<double>(ps->d, ps->push.d, s)
                                                 : launch_push_gather<float>(ps->d, ps->push.d, s);
    if (e != hipSuccess) return kErrHip;
  }
  return kOk;
}

// Rows per lane group of the static multi-RHS kernel: the configured value,
// else 4 when a row takes 8 or more lanes (chunks of 32 or fewer rows), 2 at
// 4 lanes, 1 below (chunks already 32 or 64 rows).
int multi_rows(const Config& c, int lanes_per_row) {
  (void)lanes_per_row;
  // default 1: it was the fastest choice for every column count and pattern
  // measured (2 to 16 columns, meshes and ILU(0) factors)
  return c.mrows == 2 || c.mrows == 4 ? c.mrows : 1;
}

// Column-wise solve, one right-hand side: LEVC (a launch per level) or SLFC
// (one persistent launch, chunk c on wavefront c mod W, or by XCD region).
template <typename T>
int solve_column(sptrsv_handle_t h, PlanState& ps, const Config& c, const void* b, void* x,
                 hipStream_t s, const SolveExt& ext) {
  if (!ps.push.built) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) return kErrHip;
    if (cap != hipStreamCaptureStatusNone || ext.no_alloc) return kErrNotSupported;
    if (const int st = build_push_state(h, ps, s)) return st;
  }
  int err = kOk;
  ChunkEntry* ch = get_push_chunks(ps, c.group, c.epl, &err, ext.no_alloc);
  if (!ch) return err;
  ColumnArgs a;
  a.plan = &ps.d;
  a.push = &ps.push.d;
  a.chunks = &ch->d;
  a.b = b;
  a.x = x;
  a.acc = h->col_acc;
  a.cnt = h->col_cnt;
  a.status = h->scratch.status;
  a.arrive = h->scratch.arrive;
  a.res_limit = h->res_limit;
  a.coop = h->coop;
  a.spin_limit = h->spin_limit;
  a.wg = h->wg;
  if (launch_column_init<T>(a, s) != hipSuccess) return kErrHip;
  hipEvent_t stop;
  if (c.algo == SPTRSV_ALGO_COLUMN_LEVEL) {
    timing_begin(h, s, &stop, ext.no_alloc);
    for (int m = 0; m < ps.h.nlev; ++m)
      if (launch_column_level<T>(a, ch->level_chunk[m], ch->level_chunk[m + 1], s) != hipSuccess)
        return kErrHip;
    timing_end(s, stop);
    return kOk;
  }
  a.grid = persistent_grid(h, 4, c.grid, ch->d.count);
  const int W = a.grid * (h->wg / 64);
  const int wpb = h->wg / 64;
  const int regions = (c.assign == SPTRSV_ASSIGN_XCD && W % (8 * wpb) == 0) ? 8 : 1;
  const WaveLists* wl = get_wave_lists(*ch, W, regions, wpb, &err, ext.no_alloc);
  if (!wl) return err;
  a.wave_ptr = wl->ptr;
  a.wave_list = wl->list;
  timing_begin(h, s, &stop, ext.no_alloc);
  if (launch_column_self<T>(a, s) != hipSuccess) return kErrHip;
  timing_end(s, stop);
  return kOk;
}

template <typename T>
int solve_impl(sptrsv_handle_t h, PlanState& ps, const Config& c_in, const void* b, void* x,
               int nrhs, int ld, hipStream_t s, const SolveExt& ext = SolveExt()) {
  const int n = h->n;
  h->last_stream = s;
  if (n == 0 || nrhs == 0) return kOk;
  const bool multi = nrhs > 1;
  if (is_column(c_in.algo) && !multi) return solve_column<T>(h, ps, c_in, b, x, s, ext);
  // several right-hand sides under a column-wise schedule: row-wise, self-scheduled
  Config c = c_in;
  if (is_column(c.algo)) {
    c.algo = SPTRSV_ALGO_SELF;
    c.sync = SPTRSV_SYNC_VALUE;
  }
  int kl = 1;
  while (kl < nrhs && kl < 64) kl <<= 1;
  int err = kOk;
  // static assignment keeps one row per lane (its pipeline holds one row)
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess) return kErrHip;
  const bool capturing = cap != hipStreamCaptureStatusNone;
  bool use_static = c.algo == SPTRSV_ALGO_SELF && (multi || c.sync == SPTRSV_SYNC_VALUE) &&
                    (c.assign == SPTRSV_ASSIGN_STATIC || c.assign == SPTRSV_ASSIGN_XCD);
  // several right-hand sides, static: each lane group owns mrows rows
  const int mrows = multi && use_static ? multi_rows(c, kl) : 1;
  ChunkEntry* ch = multi ? get_chunks(h, ps, 0, 0, 64 / kl, mrows, &err, ext.no_alloc)
                         : get_chunks(h, ps, c.group, c.epl, 0, use_static ? 1 : c.rpl, &err,
                                      ext.no_alloc);
  if (!ch) return err;
  // under capture (or without allocation) the per-wavefront lists cannot be
  // uploaded: the static form is used only when they exist
  // (sptrsv_graph_capture and the analysis build them), else the ticket form
  if (use_static && (capturing || ext.no_alloc) &&
      !static_lists_ready(h, *ch, c, multi ? mrows : 0)) {
    use_static = false;
    if (multi ? mrows != 1 && !(ch = get_chunks(h, ps, 0, 0, 64 / kl, 1, &err, ext.no_alloc))
              : c.rpl != 1 &&
                    !(ch = get_chunks(h, ps, c.group, c.epl, 0, c.rpl, &err, ext.no_alloc)))
      return err;
  }
  // the static schedules with one right-hand side may space the values out
  const int stride = use_static && !multi ? c.stride : 1;
  const int64_t xp_need = static_cast<int64_t>(n) * nrhs * stride;
  void* xp = ext.xp;
  if (xp) {
    if (xp_need * static_cast<int64_t>(h->vb) > ext.xp_bytes) return kErrTooLarge;
  } else {
    if ((err = ensure_xp(h, xp_need))) return err;
    xp = h->xp;
  }
  if (multi) {
    if (ext.no_alloc) return kErrNotSupported;
    if ((err = ensure_multi(h, ps, xp_need, s))) return err;
  }
  SolveArgs a;
  a.plan = &ps.d;
  a.chunks = &ch->d;
  a.scratch = h->scratch;
  a.b = b;
  a.x = x;
  a.xp = xp;
  a.bp = multi ? h->bp : nullptr;
  a.nrhs = nrhs;
  a.ld = ld;
  a.spin_limit = h->spin_limit;
  a.poll = c.poll;
  a.xp_stride = stride;
  a.res_limit = h->res_limit;
  a.coop = h->coop;
  a.mrows = use_static ? mrows : 1;
  a.wg = h->wg;
  hipEvent_t stop;
  if (c.algo == SPTRSV_ALGO_BLOCK && !multi) {
    const int dir = (&ps == &h->trn) ? 1 : 0;
    BlockState& bs = h->blk[dir];
    if (!bs.built) return ext.no_alloc ? kErrNotSupported : kErrInvalidArg;
    a.plan = &bs.ps.d;
    int threads = 64;
    while (threads < bs.info.max_level && threads < 1024) threads <<= 1;
    const size_t lds_bytes = static_cast<size_t>(bs.info.max_rows) * sizeof(T);
    const int lds_rows = lds_bytes <= static_cast<size_t>(h->lds_limit) ? bs.info.max_rows : 0;
    const int nseg = static_cast<int>(bs.info.seg_row0.size()) - 1;
    // whole systems in LDS when they fit and one wavefront takes every level
    // (with wider levels the streamed kernel's barrier loop was faster)
    const bool resident = h->block_resident && bs.res_bytes > 0 &&
                          bs.res_bytes <= h->lds_limit && bs.info.max_level <= 64;
    timing_begin(h, s, &stop, ext.no_alloc);
    const hipError_t le =
        resident ? launch_block_res<T>(a, bs.seg_base, bs.lev_pos, nseg, kResidentThreads,
                                       static_cast<int>(bs.res_bytes), s)
                 : launch_block<T>(a, bs.seg_row0, bs.seg_base, bs.lev_pos, nseg, threads,
                                   lds_rows, s);
    if (le != hipSuccess) return kErrHip;
    timing_end(s, stop);
    return kOk;
  }
  // several right-hand sides: B into position order (and xp filled with the
  // readiness sentinel for the value-synchronised solves), X out afterwards
  const bool level = c.algo == SPTRSV_ALGO_LEVEL || c.algo == SPTRSV_ALGO_BLOCK;
  if (multi && launch_multi_in<T>(n, nrhs, ld, static_cast<const T*>(b), ps.d.row_pos,
                                  static_cast<T*>(h->bp), static_cast<T*>(xp), !level,
                                  h->scratch.arrive, s) != hipSuccess)
    return kErrHip;
  auto multi_out = [&]() {
    return !multi || launch_multi_out<T>(n, nrhs, ld, static_cast<const T*>(xp), ps.d.row_pos,
                                         static_cast<T*>(x), s) == hipSuccess
               ? kOk
               : kErrHip;
  };
  if (level) {
    timing_begin(h, s, &stop, ext.no_alloc);
    // one lane per row everywhere and one right-hand side: a thread per row,
    // straight from the level's position range
    const bool flat = !multi && ch->max_lg == 0;
    for (int m = 0; m < ps.h.nlev; ++m) {
      const hipError_t e =
          flat ? launch_level_flat<T>(a, ps.h.pos_ilev[m], ps.h.pos_ilev[m + 1], s)
               : launch_level<T>(a, ch->level_chunk[m], ch->level_chunk[m + 1], s);
      if (e != hipSuccess) return kErrHip;
    }
    timing_end(s, stop);
    return multi_out();
  }
  if (c.algo != SPTRSV_ALGO_SELF) return kErrNotSupported;
  if (c.sync == SPTRSV_SYNC_FLAG && !multi) {
    a.grid = persistent_grid(h, 1, c.grid, ch->d.count);
    timing_begin(h, s, &stop, ext.no_alloc);
    if (launch_self_flag<T>(a, s) != hipSuccess) return kErrHip;
    timing_end(s, stop);
    return kOk;
  }
  // value sync: xp starts as the sentinel (b == x needs no copy: a row reads
  // its own b before any write of its own x, and x is only written)
  if (!multi &&
      launch_fill_sentinel<T>(static_cast<T*>(xp), xp_need, h->scratch.arrive, s) != hipSuccess)
    return kErrHip;
  a.grid = persistent_grid(h, use_static ? multi_kind(multi ? mrows : 0) : 0, c.grid,
                           ch->d.count);
  if (use_static) {
    const WaveLists* wl = static_lists(h, *ch, c, &err, multi ? mrows : 0);
    if (!wl) return err;
    a.wave_ptr = wl->ptr;
    a.wave_list = wl->list;
  }
  timing_begin(h, s, &stop, ext.no_alloc);
  const hipError_t e = use_static ? launch_self_static<T>(a, s) : launch_self_value<T>(a, s);
  if (e != hipSuccess) return kErrHip;
  timing_end(s, stop);
  return multi_out();
}

// Work on a handle's buffers (its position-ordered solution, flags,
// counters, gathered values) issued on a different stream than the previous
// such work first waits for that work: the library records an event after
// each, so calls on several streams are serialized instead of racing.  Under
// graph capture nothing is recorded or waited for (the capturing stream
// orders the graph; the caller orders graph launches).
int order_begin(sptrsv_handle_t h, hipStream_t s, bool* capturing) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess) return kErrHip;
  *capturing = cap != hipStreamCaptureStatusNone;
  if (*capturing || !h->order_pending || h->order_stream == s) return kOk;
  HIPCHK(hipStreamWaitEvent(s, h->order_ev, 0));
  return kOk;
}

int order_end(sptrsv_handle_t h, hipStream_t s, bool capturing) {
  if (capturing) return kOk;
  if (!h->order_ev) HIPCHK(hipEventCreateWithFlags(&h->order_ev, hipEventDisableTiming));
  HIPCHK(hipEventRecord(h->order_ev, s));
  h->order_stream = s;
  h->order_pending = true;
  return kOk;
}

int solve_dispatch_ordered(sptrsv_handle_t h, bool transpose, const void* b, void* x, int nrhs,
                           int ld, hipStream_t s, const SolveExt& ext);

int solve_dispatch(sptrsv_handle_t h, bool transpose, const void* b, void* x, int nrhs, int ld,
                   hipStream_t s, const SolveExt& ext = SolveExt()) {
  if (!h) return kErrInvalidArg;
  if (h->n > 0 && (!b || !x)) return kErrInvalidArg;
  bool capturing = false;
  int st = order_begin(h, s, &capturing);
  if (st) return st;
  st = solve_dispatch_ordered(h, transpose, b, x, nrhs, ld, s, ext);
  const int st2 = order_end(h, s, capturing);
  return st ? st : st2;
}

// Several right-hand sides on a pattern the multi-RHS kernels do not suit
// (rows longer than 64 entries), static schedule: all columns in one launch
// of the one-RHS static kernel over a column-batched chunk table.  Column q
// reads b + q ld, publishes into its own slice of the position-ordered
// solution (n slots apart) and writes x + q ld; each column is chunked and
// summed exactly as sptrsv_solve on it.
template <typename T>
int solve_columns(sptrsv_handle_t h, PlanState& ps, const Config& c_in, const void* b, void* x,
                  int nrhs, int ld, hipStream_t s, const SolveExt& ext) {
  const int n = h->n;
  // grid left unset: 4 wavefronts per CU from 8 columns, else 2 (power-law
  // 10^6, 16 columns: 3.25 ms at 4 per CU, 3.77 at 8; 4 columns: 1.42 / 1.44
  // ms at 4 / 2)
  Config c = c_in;
  if (!(h->set_mask & kSetGrid)) c.grid = (nrhs >= 8 ? 4 : 2) * h->num_cu;
  h->last_stream = s;
  if (n == 0) return kOk;
  int err = kOk;
  ChunkEntry* base = get_chunks(h, ps, c.group, c.epl, 0, 1, &err);
  if (!base) return err;
  ChunkEntry* ch = get_col_chunks(ps, c.group, c.epl, nrhs, *base, &err);
  if (!ch) return err;
  const int64_t col_elems = static_cast<int64_t>(n) * c.stride;
  if ((err = ensure_xp(h, col_elems * nrhs))) return err;
  SolveArgs a;
  a.plan = &ps.d;
  a.chunks = &ch->d;
  a.scratch = h->scratch;
  a.b = b;
  a.x = x;
  a.xp = h->xp;
  a.nrhs = 1;
  a.ld = ld;
  a.spin_limit = h->spin_limit;
  a.poll = c.poll;
  a.xp_stride = c.stride;
  a.xp_col = col_elems;
  a.res_limit = h->res_limit;
  a.coop = h->coop;
  a.wg = h->wg;
  a.grid = persistent_grid(h, 3, c.grid, ch->d.count);
  const int W = a.grid * (h->wg / 64);
  const int wpb = h->wg / 64;
  const WaveLists* wl = get_wave_lists(
      *ch, W, (c.assign == SPTRSV_ASSIGN_XCD && W % (8 * wpb) == 0) ? 8 : 1, wpb, &err);
  if (!wl) return err;
  a.wave_ptr = wl->ptr;
  a.wave_list = wl->list;
  if (launch_fill_sentinel<T>(static_cast<T*>(h->xp), col_elems * nrhs, h->scratch.arrive, s) !=
      hipSuccess)
    return kErrHip;
  hipEvent_t stop;
  timing_begin(h, s, &stop, ext.no_alloc);
  if (launch_self_static<T>(a, s) != hipSuccess) return kErrHip;
  timing_end(s, stop);
  return kOk;
}

int solve_dispatch_ordered(sptrsv_handle_t h, bool transpose, const void* b, void* x, int nrhs,
                           int ld, hipStream_t s, const SolveExt& ext) {
  if (transpose && !h->trn.built) {
    if (ext.no_alloc) return kErrNotSupported;
    const int st = build_transpose(h, s);
    if (st) return st;
  }
  PlanState& ps = transpose ? h->trn : h->fwd;
  const Config c = nrhs > 1 ? resolve_multi(h, nrhs) : resolve(h);
  if (nrhs > 1 && multi_by_columns(ps, c)) {
    // each column equals sptrsv_solve on it, bit for bit: all at once with
    // the static schedule (outside a capture, with allocation), else one
    // after another
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) return kErrHip;
    if (c.algo == SPTRSV_ALGO_SELF && c.sync == SPTRSV_SYNC_VALUE &&
        (c.assign == SPTRSV_ASSIGN_STATIC || c.assign == SPTRSV_ASSIGN_XCD) && !ext.no_alloc &&
        !ext.xp && cap == hipStreamCaptureStatusNone)
      return h->dtype == SPTRSV_F64 ? solve_columns<double>(h, ps, c, b, x, nrhs, ld, s, ext)
                                    : solve_columns<float>(h, ps, c, b, x, nrhs, ld, s, ext);
    const size_t col = static_cast<size_t>(ld) * h->vb;
    for (int q = 0; q < nrhs; ++q) {
      const int st = solve_dispatch_ordered(h, transpose, static_cast<const char*>(b) + q * col,
                                            static_cast<char*>(x) + q * col, 1, h->n, s, ext);
      if (st) return st;
    }
    return kOk;
  }
  if (c.algo == SPTRSV_ALGO_BLOCK && nrhs == 1 && !h->blk[transpose ? 1 : 0].built) {
    if (ext.no_alloc) return kErrNotSupported;
    const int st = build_block(h, transpose ? 1 : 0, s);
    if (st) return st;
  }
  if (h->dtype == SPTRSV_F64) return solve_impl<double>(h, ps, c, b, x, nrhs, ld, s, ext);
  return solve_impl<float>(h, ps, c, b, x, nrhs, ld, s, ext);
}

// Builds everything solves with schedule c (one right-hand side) on T or
// T^T need, with synchronous uploads: the chunk table, the occupancy
// figures, the static schedule's per-wavefront lists and position-ordered
// buffer, the block plan, the push lists.  Run before a graph capture and at
// the end of the analysis (for the default schedule), so that later solves
// with c allocate nothing.
int prepare_schedule(sptrsv_handle_t h, bool transpose, const Config& c, hipStream_t s) {
  if (h->n == 0) return kOk;
  if (transpose)
    if (const int st = build_transpose(h, s)) return st;
  int err = kOk;
  PlanState& ps = transpose ? h->trn : h->fwd;
  if (!get_chunks(h, ps, c.group, c.epl, 0, c.rpl, &err)) return err;
  for (int kind : {0, 1, 3, 4}) (void)blocks_per_cu(h, kind);
  if (c.algo == SPTRSV_ALGO_SELF && c.sync == SPTRSV_SYNC_VALUE &&
      (c.assign == SPTRSV_ASSIGN_STATIC || c.assign == SPTRSV_ASSIGN_XCD)) {
    ChunkEntry* ch = get_chunks(h, ps, c.group, c.epl, 0, 1, &err);
    if (!ch || !static_lists(h, *ch, c, &err)) return err;
    if ((err = ensure_xp(h, static_cast<int64_t>(h->n) * c.stride))) return err;
  }
  if (c.algo == SPTRSV_ALGO_BLOCK && (err = build_block(h, transpose ? 1 : 0, s))) return err;
  if (is_column(c.algo)) {
    if ((err = build_push_state(h, ps, s))) return err;
    ChunkEntry* ch = get_push_chunks(ps, c.group, c.epl, &err);
    if (!ch) return err;
    if (c.algo == SPTRSV_ALGO_COLUMN_SELF) {
      const int grid = persistent_grid(h, 4, c.grid, ch->d.count);
      const int W = grid * (h->wg / 64);
      const int wpb = h->wg / 64;
      if (!get_wave_lists(*ch, W, (c.assign == SPTRSV_ASSIGN_XCD && W % (8 * wpb) == 0) ? 8 : 1,
                          wpb, &err))
        return err;
    }
  }
  return kOk;
}

int init_handle_common(sptrsv_handle_t h, hipStream_t s) {
  (void)hipGetDevice(&h->device);
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess &&
      ncu > 0)
    h->num_cu = ncu;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) ==
          hipSuccess &&
      lds > 0)
    h->lds_limit = lds;
  // a kernel may opt in to more than the default per-workgroup LDS
  int optin = 0;
  if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, h->device) ==
          hipSuccess &&
      optin > h->lds_limit)
    h->lds_limit = optin;
  int err = kOk;
  h->scratch.ticket = dalloc<int>(1, &err);
  h->scratch.status = dalloc<int>(1, &err);
  h->scratch.epoch = dalloc<unsigned>(1, &err);
  h->scratch.flags = dalloc<unsigned>(h->n, &err);
  h->scratch.arrive = dalloc<int>(1, &err);
  if (err) return err;
  if ((err = ensure_xp(h, h->n))) return err;
  HIPCHK(hipEventCreateWithFlags(&h->order_ev, hipEventDisableTiming));
  HIPCHK(launch_init_scratch(h->scratch, h->n, s));
  return kOk;
}

// Validation, analysis and upload of the forward plan from a host pattern.
int analyze_from_host(sptrsv_handle_t h, const void* vals, hipStream_t s) {
  int st = validate_pattern(h->n, h->nnz, h->rp_h.data(), h->col_h.data(), h->upper, h->unit,
                            nullptr);
  if (st) return st;
  build_plan(h->n, h->rp_h.data(), h->col_h.data(), nullptr, h->upper, h->unit, h->fwd.h);
  if ((st = init_handle_common(h, s))) return st;
  if ((st = upload_plan(h->fwd, h->vb, s))) return st;
  if ((st = gather(h, h->fwd, vals, s))) return st;
  return read_status(h, s, true);
}

// Takes over the arrays of a device analysis as plan ps (the host plan keeps
// nlev, ilev and off_ptr; the rest is downloaded only if the host needs it)
// and allocates its value buffer.
int install_device_plan(sptrsv_handle_t h, PlanState& ps, DeviceAnalysis& da, bool upper) {
  HostPlan& p = ps.h;
  p = HostPlan();
  p.n = h->n;
  p.nlev = da.nlev;
  p.nnz = h->nnz;
  p.noff = da.noff;
  p.upper = upper;
  p.unit_diag = h->unit;
  p.ilev = std::move(da.ilev);
  p.pos_ilev = p.ilev;
  p.off_ptr = std::move(da.off_ptr_h);
  p.max_row_len = da.max_row_len;
  DevPlan& d = ps.d;
  d = DevPlan();
  d.n = h->n;
  d.nlev = da.nlev;
  d.noff = da.noff;
  d.off_ptr = da.off_ptr;
  d.off_col = da.off_col;
  d.off_pos = da.off_pos;
  d.off_src = da.off_src;
  d.diag_src = da.diag_src;
  d.pos_row = da.pos_row;
  ps.a_level = da.level;
  ps.a_depcnt = da.depcnt;
  ps.a_jlev = da.jlev;
  ps.host_complete = false;
  da = DeviceAnalysis();        // the plan owns the arrays now
  int err = kOk;
  ps.vals_buf =
      dalloc<char>((static_cast<size_t>(d.noff) + 2 * static_cast<size_t>(h->n)) * h->vb, &err);
  if (!ps.vals_buf) return err;
  d.off_val = ps.vals_buf;
  d.diag = static_cast<char*>(ps.vals_buf) + static_cast<size_t>(d.noff) * h->vb;
  d.dinv = static_cast<char*>(d.diag) + static_cast<size_t>(h->n) * h->vb;
  ps.built = true;
  return kOk;
}

// Setup on the device (levels, level-ordered layout) from the caller's device
// pattern; the plan stays on the device, only nlev, ilev and off_ptr come to
// the host (for the chunk tables).  Returns kErrNotSupported for a pattern
// the device route does not take; the caller then runs the host route.
int analyze_on_device(sptrsv_handle_t h, const int* row_ptr, const int* col_idx, const void* vals,
                      hipStream_t s, bool copy_pattern = true) {
  (void)hipGetDevice(&h->device);
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess &&
      ncu > 0)
    h->num_cu = ncu;
  DeviceAnalysis da;
  int st = device_analysis(h->n, h->nnz, row_ptr, col_idx, h->upper, h->unit, h->num_cu, s, da);
  if (st) return st;
  if ((st = install_device_plan(h, h->fwd, da, h->upper))) {
    free_device_analysis(da);
    return st;
  }
  int err = kOk;
  // the handle's own copy of the pattern, for what is built later (a
  // batched handle's concatenation already is its own)
  h->pattern_host = false;
  if (!copy_pattern) {
    h->rp_dev = const_cast<int*>(row_ptr);
    h->col_dev = const_cast<int*>(col_idx);
  } else {
    h->rp_dev = dalloc<int>(static_cast<size_t>(h->n) + 1, &err);
    h->col_dev = dalloc<int>(static_cast<size_t>(h->nnz), &err);
    if (err) return err;
    HIPCHK(hipMemcpyAsync(h->rp_dev, row_ptr, (static_cast<size_t>(h->n) + 1) * sizeof(int),
                          hipMemcpyDeviceToDevice, s));
    if (h->nnz > 0)
      HIPCHK(hipMemcpyAsync(h->col_dev, col_idx, static_cast<size_t>(h->nnz) * sizeof(int),
                            hipMemcpyDeviceToDevice, s));
  }
  if ((st = init_handle_common(h, s))) return st;
  if ((st = gather(h, h->fwd, vals, s))) return st;
  return read_status(h, s, true);
}

void free_block(BlockState& b) {
  free_plan(b.ps);
  dfree(b.seg_row0);
  dfree(b.seg_base);
  dfree(b.lev_pos);
  b = BlockState();
}

void destroy_handle(sptrsv_handle_t h) {
  if (!h) return;
  if (h->order_ev) (void)hipEventDestroy(h->order_ev);
  free_plan(h->fwd);
  free_plan(h->trn);
  free_block(h->blk[0]);
  free_block(h->blk[1]);
  dfree(h->scratch.ticket);
  dfree(h->scratch.status);
  dfree(h->scratch.epoch);
  dfree(h->scratch.flags);
  dfree(h->scratch.arrive);
  h->xp_buf.reset();
  h->xp = nullptr;
  dfree(h->bp);
  dfree(h->rp_cat);
  dfree(h->col_cat);
  dfree(h->vals_cat);
  if (h->rp_dev != h->rp_cat) dfree(h->rp_dev);
  if (h->col_dev != h->col_cat) dfree(h->col_dev);
  dfree(h->col_acc);
  dfree(h->col_cnt);
  for (auto& pr : h->ev_pool) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  delete h;
}

}  // namespace

namespace sptrsv {

int solve_external_scratch(sptrsv_handle_t h, const void* b, void* x, void* xp, int64_t xp_bytes,
                           hipStream_t s) {
  if (!h || !xp || xp_bytes <= 0) return kErrInvalidArg;
  SolveExt ext;
  ext.xp = xp;
  ext.xp_bytes = xp_bytes;
  ext.no_alloc = true;
  return solve_dispatch(h, false, b, x, 1, h->n, s, ext);
}

int handle_device(sptrsv_handle_t h) { return h ? h->device : -1; }

}  // namespace sptrsv

extern "C" {

int sptrsv_analyze_ex(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                      const void* vals, sptrsv_dtype dtype, sptrsv_uplo uplo, int unit_diag,
                      int setup, hipStream_t stream, sptrsv_handle_t* out) {
  if (!out) return kErrInvalidArg;
  *out = nullptr;
  if (n < 0 || nnz < 0 || (dtype != SPTRSV_F64 && dtype != SPTRSV_F32) ||
      (uplo != SPTRSV_LOWER && uplo != SPTRSV_UPPER) ||
      (setup != SPTRSV_SETUP_HOST && setup != SPTRSV_SETUP_DEVICE))
    return kErrInvalidArg;
  if (!row_ptr || (nnz > 0 && (!col_idx || !vals))) return kErrInvalidArg;
  const auto t0 = std::chrono::steady_clock::now();
  auto fresh = [&]() {
    sptrsv_handle_t h = new (std::nothrow) sptrsv_handle_s;
    if (!h) return h;
    h->n = n;
    h->nnz = nnz;
    h->dtype = dtype;
    h->vb = dtype == SPTRSV_F64 ? 8 : 4;
    h->upper = uplo == SPTRSV_UPPER;
    h->unit = unit_diag != 0;
    return h;
  };
  sptrsv_handle_t h = fresh();
  if (!h) return kErrOom;
  int st = kErrNotSupported;
  if (setup == SPTRSV_SETUP_DEVICE && n > 0) {
    st = analyze_on_device(h, row_ptr, col_idx, vals, stream);
    if (st == kOk) h->setup = SPTRSV_SETUP_DEVICE;
    if (st == kErrNotSupported) {
      // the host route decides (and reports the exact validation error)
      destroy_handle(h);
      if (!(h = fresh())) return kErrOom;
    }
  }
  if (st == kErrNotSupported) {
    h->rp_h.resize(static_cast<size_t>(n) + 1);
    h->col_h.resize(nnz);
    if (hipMemcpyAsync(h->rp_h.data(), row_ptr, (static_cast<size_t>(n) + 1) * sizeof(int),
                       hipMemcpyDeviceToHost, stream) != hipSuccess ||
        (nnz > 0 && hipMemcpyAsync(h->col_h.data(), col_idx, static_cast<size_t>(nnz) * sizeof(int),
                                   hipMemcpyDeviceToHost, stream) != hipSuccess) ||
        hipStreamSynchronize(stream) != hipSuccess) {
      destroy_handle(h);
      return kErrHip;
    }
    st = analyze_from_host(h, vals, stream);
    h->setup = SPTRSV_SETUP_HOST;
  }
  // the default schedule's work tables, so that the first solve allocates nothing
  if (!st) st = prepare_schedule(h, false, resolve(h), stream);
  if (st) {
    destroy_handle(h);
    return st;
  }
  h->setup_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = h;
  return kOk;
}

int sptrsv_analyze(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                   const void* vals, sptrsv_dtype dtype, sptrsv_uplo uplo, int unit_diag,
                   hipStream_t stream, sptrsv_handle_t* out) {
  return sptrsv_analyze_ex(n, nnz, row_ptr, col_idx, vals, dtype, uplo, unit_diag,
                           SPTRSV_SETUP_HOST, stream, out);
}

int sptrsv_get_setup(sptrsv_handle_t h, int32_t* route, double* ms) {
  if (!h) return kErrInvalidArg;
  if (route) *route = h->setup;
  if (ms) *ms = h->setup_ms;
  return kOk;
}

int sptrsv_analyze_batched_ex(int32_t count, const int32_t* n, const int32_t* nnz,
                              const int32_t* const* row_ptr, const int32_t* const* col_idx,
                              const void* const* vals, sptrsv_dtype dtype, sptrsv_uplo uplo,
                              int unit_diag, int setup, hipStream_t stream, sptrsv_handle_t* out) {
  if (!out) return kErrInvalidArg;
  *out = nullptr;
  if (count < 1 || !n || !nnz || !row_ptr || !col_idx || !vals ||
      (dtype != SPTRSV_F64 && dtype != SPTRSV_F32) || (uplo != SPTRSV_LOWER && uplo != SPTRSV_UPPER) ||
      (setup != SPTRSV_SETUP_HOST && setup != SPTRSV_SETUP_DEVICE))
    return kErrInvalidArg;
  int64_t ntot = 0, nnztot = 0;
  for (int s = 0; s < count; ++s) {
    if (n[s] < 0 || nnz[s] < 0 || !row_ptr[s] || (nnz[s] > 0 && (!col_idx[s] || !vals[s])))
      return kErrInvalidArg;
    ntot += n[s];
    nnztot += nnz[s];
  }
  if (ntot > INT32_MAX || nnztot > INT32_MAX) return kErrInvalidArg;
  const auto t0 = std::chrono::steady_clock::now();
  if (setup == SPTRSV_SETUP_DEVICE && ntot > 0) {
    // concatenation and analysis in device memory; a pattern this route
    // does not take (or an invalid one) goes to the host route below
    sptrsv_handle_t h = new (std::nothrow) sptrsv_handle_s;
    if (!h) return kErrOom;
    h->n = static_cast<int>(ntot);
    h->nnz = nnztot;
    h->dtype = dtype;
    h->vb = dtype == SPTRSV_F64 ? 8 : 4;
    h->upper = uplo == SPTRSV_UPPER;
    h->unit = unit_diag != 0;
    h->batched = true;
    h->sys_n.assign(n, n + count);
    h->sys_nnz.assign(nnz, nnz + count);
    int err = kOk;
    h->rp_cat = dalloc<int>(static_cast<size_t>(ntot) + 1, &err);
    h->col_cat = dalloc<int>(static_cast<size_t>(nnztot), &err);
    h->vals_cat = dalloc<char>(static_cast<size_t>(nnztot) * h->vb, &err);
    int st = err;
    if (!st) {
      std::vector<ConcatSystem> sys(count);
      for (int k = 0; k < count; ++k) sys[k] = ConcatSystem{row_ptr[k], col_idx[k], vals[k], n[k], nnz[k]};
      st = device_concat(sys, static_cast<int>(h->vb), h->rp_cat, h->col_cat, h->vals_cat, stream);
    }
    if (!st) st = analyze_on_device(h, h->rp_cat, h->col_cat, h->vals_cat, stream, false);
    if (!st) st = prepare_schedule(h, false, resolve(h), stream);
    if (!st && hipStreamSynchronize(stream) != hipSuccess) st = kErrHip;
    if (!st) {
      h->setup = SPTRSV_SETUP_DEVICE;
      h->setup_ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      *out = h;
      return kOk;
    }
    destroy_handle(h);
    if (st != kErrNotSupported) return st;
  }
  sptrsv_handle_t h = new (std::nothrow) sptrsv_handle_s;
  if (!h) return kErrOom;
  h->n = static_cast<int>(ntot);
  h->nnz = nnztot;
  h->dtype = dtype;
  h->vb = dtype == SPTRSV_F64 ? 8 : 4;
  h->upper = uplo == SPTRSV_UPPER;
  h->unit = unit_diag != 0;
  h->batched = true;
  h->sys_n.assign(n, n + count);
  h->sys_nnz.assign(nnz, nnz + count);
  h->rp_h.assign(static_cast<size_t>(ntot) + 1, 0);
  h->col_h.resize(nnztot);
  int err = kOk;
  h->vals_cat = dalloc<char>(static_cast<size_t>(nnztot) * h->vb, &err);
  if (err) {
    destroy_handle(h);
    return err;
  }
  int64_t roff = 0, eoff = 0;
  std::vector<int> rp_tmp;
  for (int s = 0; s < count; ++s) {
    rp_tmp.resize(static_cast<size_t>(n[s]) + 1);
    if (hipMemcpyAsync(rp_tmp.data(), row_ptr[s], rp_tmp.size() * sizeof(int),
                       hipMemcpyDeviceToHost, stream) != hipSuccess ||
        (nnz[s] > 0 &&
         (hipMemcpyAsync(h->col_h.data() + eoff, col_idx[s], static_cast<size_t>(nnz[s]) * sizeof(int),
                         hipMemcpyDeviceToHost, stream) != hipSuccess ||
          hipMemcpyAsync(static_cast<char*>(h->vals_cat) + eoff * h->vb, vals[s],
                         static_cast<size_t>(nnz[s]) * h->vb, hipMemcpyDeviceToDevice,
                         stream) != hipSuccess)) ||
        hipStreamSynchronize(stream) != hipSuccess) {
      destroy_handle(h);
      return kErrHip;
    }
    // each system is validated on its own (its errors are its own)
    const int st = validate_pattern(n[s], nnz[s], rp_tmp.data(), h->col_h.data() + eoff,
                                    h->upper, h->unit, nullptr);
    if (st) {
      destroy_handle(h);
      return st;
    }
    for (int i = 0; i < n[s]; ++i) h->rp_h[roff + i + 1] = static_cast<int>(rp_tmp[i + 1] + eoff);
    for (int64_t k = eoff; k < eoff + nnz[s]; ++k) h->col_h[k] += static_cast<int>(roff);
    roff += n[s];
    eoff += nnz[s];
  }
  int st = analyze_from_host(h, h->vals_cat, stream);
  if (!st) st = upload_ints(&h->rp_cat, h->rp_h, stream);
  if (!st) st = upload_ints(&h->col_cat, h->col_h, stream);
  if (!st) st = prepare_schedule(h, false, resolve(h), stream);
  if (!st && hipStreamSynchronize(stream) != hipSuccess) st = kErrHip;
  if (st) {
    destroy_handle(h);
    return st;
  }
  h->setup = SPTRSV_SETUP_HOST;
  h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = h;
  return kOk;
}

int sptrsv_analyze_batched(int32_t count, const int32_t* n, const int32_t* nnz,
                           const int32_t* const* row_ptr, const int32_t* const* col_idx,
                           const void* const* vals, sptrsv_dtype dtype, sptrsv_uplo uplo,
                           int unit_diag, hipStream_t stream, sptrsv_handle_t* out) {
  return sptrsv_analyze_batched_ex(count, n, nnz, row_ptr, col_idx, vals, dtype, uplo, unit_diag,
                                   SPTRSV_SETUP_HOST, stream, out);
}

int sptrsv_update_values(sptrsv_handle_t h, const void* vals, hipStream_t stream) {
  if (!h || (h->nnz > 0 && !vals)) return kErrInvalidArg;
  if (h->batched) return kErrInvalidArg;
  bool capturing = false;
  int st = order_begin(h, stream, &capturing);
  if (st) return st;
  st = gather(h, h->fwd, vals, stream);
  if (!st && h->trn.built) st = gather(h, h->trn, h->fwd.vals_buf, stream);
  if (!st && h->blk[0].built) st = gather(h, h->blk[0].ps, h->fwd.vals_buf, stream);
  if (!st && h->blk[1].built) st = gather(h, h->blk[1].ps, h->trn.vals_buf, stream);
  if (!st) st = regather_push(h, stream);
  h->last_stream = stream;
  const int st2 = order_end(h, stream, capturing);
  return st ? st : st2;
}

int sptrsv_update_values_batched(sptrsv_handle_t h, const void* const* vals, hipStream_t stream) {
  if (!h || !vals || !h->batched) return kErrInvalidArg;
  for (size_t s = 0; s < h->sys_n.size(); ++s)
    if (h->sys_nnz[s] > 0 && !vals[s]) return kErrInvalidArg;
  bool capturing = false;
  if (const int st0 = order_begin(h, stream, &capturing)) return st0;
  int st = kOk;
  int64_t eoff = 0;
  for (size_t s = 0; s < h->sys_n.size() && !st; ++s) {
    if (h->sys_nnz[s] > 0 &&
        hipMemcpyAsync(static_cast<char*>(h->vals_cat) + eoff * h->vb, vals[s],
                       static_cast<size_t>(h->sys_nnz[s]) * h->vb, hipMemcpyDeviceToDevice,
                       stream) != hipSuccess)
      st = kErrHip;
    eoff += h->sys_nnz[s];
  }
  if (!st) st = gather(h, h->fwd, h->vals_cat, stream);
  if (!st && h->trn.built) st = gather(h, h->trn, h->fwd.vals_buf, stream);
  if (!st && h->blk[0].built) st = gather(h, h->blk[0].ps, h->fwd.vals_buf, stream);
  if (!st && h->blk[1].built) st = gather(h, h->blk[1].ps, h->trn.vals_buf, stream);
  if (!st) st = regather_push(h, stream);
  h->last_stream = stream;
  const int st2 = order_end(h, stream, capturing);
  return st ? st : st2;
}

int sptrsv_solve(sptrsv_handle_t h, const void* b, void* x, hipStream_t stream) {
  return solve_dispatch(h, false, b, x, 1, h ? h->n : 0, stream);
}

int sptrsv_solve_transpose(sptrsv_handle_t h, const void* b, void* x, hipStream_t stream) {
  return solve_dispatch(h, true, b, x, 1, h ? h->n : 0, stream);
}

int sptrsv_prepare_transpose(sptrsv_handle_t h, hipStream_t stream) {
  if (!h) return kErrInvalidArg;
  return build_transpose(h, stream);
}

int sptrsv_solve_multi(sptrsv_handle_t h, int32_t nrhs, int32_t ld, const void* B, void* X,
                       int transpose, hipStream_t stream) {
  if (!h || nrhs < 1 || ld < h->n || ld < 1) return kErrInvalidArg;
  return solve_dispatch(h, transpose != 0, B, X, nrhs, ld, stream);
}

int sptrsv_grad_vals(sptrsv_handle_t h, const int32_t* row_ptr, const int32_t* col_idx,
                     const void* grad_b, const void* x, void* grad_vals, hipStream_t stream) {
  if (!h) return kErrInvalidArg;
  if (h->n == 0) return kOk;
  if (h->batched) {
    row_ptr = h->rp_cat;
    col_idx = h->col_cat;
  }
  if (!row_ptr || (h->nnz > 0 && (!col_idx || !grad_b || !x || !grad_vals))) return kErrInvalidArg;
  hipError_t e;
  if (h->dtype == SPTRSV_F64)
    e = launch_grad_vals<double>(h->n, row_ptr, col_idx, h->unit, static_cast<const double*>(grad_b),
                                 static_cast<const double*>(x), static_cast<double*>(grad_vals),
                                 stream);
  else
    e = launch_grad_vals<float>(h->n, row_ptr, col_idx, h->unit, static_cast<const float*>(grad_b),
                                static_cast<const float*>(x), static_cast<float*>(grad_vals), stream);
  h->last_stream = stream;
  return e == hipSuccess ? kOk : kErrHip;
}

int sptrsv_set_option(sptrsv_handle_t h, sptrsv_option key, int64_t v) {
  if (!h) return kErrInvalidArg;
  if (key == SPTRSV_OPT_ALGO || key == SPTRSV_OPT_GROUP || key == SPTRSV_OPT_ENTRIES_PER_LANE ||
      key == SPTRSV_OPT_SYNC || key == SPTRSV_OPT_ROWS_PER_LANE || key == SPTRSV_OPT_GRID ||
      key == SPTRSV_OPT_ASSIGN || key == SPTRSV_OPT_POLL || key == SPTRSV_OPT_XP_STRIDE ||
      key == SPTRSV_OPT_MULTI_ROWS) {
    h->tuned = false;   // an explicit schedule option overrides the tuner's choice
    h->tuned_multi.clear();
  }
  switch (key) {
    case SPTRSV_OPT_ALGO:
      if (v != SPTRSV_ALGO_AUTO && v != SPTRSV_ALGO_LEVEL && v != SPTRSV_ALGO_SELF &&
          v != SPTRSV_ALGO_BLOCK && !is_column(static_cast<int>(v)))
        return kErrInvalidArg;
      h->algo = static_cast<int>(v);
      return kOk;
    case SPTRSV_OPT_GROUP:
      if (v < 0 || v > 64 || (v & (v - 1))) return kErrInvalidArg;
      h->group = static_cast<int>(v);
      return kOk;
    case SPTRSV_OPT_ENTRIES_PER_LANE:
      if (v < 1 || v > 4096) return kErrInvalidArg;
      h->epl = static_cast<int>(v);
      return kOk;
    case SPTRSV_OPT_SYNC:
      if (v != SPTRSV_SYNC_VALUE && v != SPTRSV_SYNC_FLAG) return kErrInvalidArg;
      h->sync = static_cast<int>(v);
      return kOk;
    case SPTRSV_OPT_SPIN_LIMIT:
      if (v < 1 || v > INT32_MAX) return kErrInvalidArg;
      h->spin_limit = static_cast<int>(v);
      return kOk;
    case SPTRSV_OPT_GRID:
      if (v < 0 || v > (1 << 20)) return kErrInvalidArg;
      h->grid = static_cast<int>(v);
      h->set_mask |= kSetGrid;
      return kOk;
    case SPTRSV_OPT_TIMING:
      h->timing = v != 0;
      return kOk;
    case SPTRSV_OPT_WG:
      if (v < 64 || v > 256 || (v % 64)) return kErrInvalidArg;
      h->wg = static_cast<int>(v);
      return kOk;
    case SPTRSV_OPT_ROWS_PER_LANE:
      if (v < 1 || v > kMaxRowsPerLane) return kErrInvalidArg;
      h->rpl = static_cast<int>(v);
      return kOk;
    case SPTRSV_OPT_ASSIGN:
      if (v != SPTRSV_ASSIGN_STATIC && v != SPTRSV_ASSIGN_TICKET && v != SPTRSV_ASSIGN_XCD)
        return kErrInvalidArg;
      h->assign = static_cast<int>(v);
      h->set_mask |= kSetAssign;
      return kOk;
    case SPTRSV_OPT_POLL:
      if (v != 0 && v != 1) return kErrInvalidArg;
      h->poll = static_cast<int>(v);
      return kOk;
    case SPTRSV_OPT_XP_STRIDE:
      if (v != 1 && v != 2 && v != 4 && v != 8 && v != 16) return kErrInvalidArg;
      h->xp_stride = static_cast<int>(v);
      h->set_mask |= kSetStride;
      return kOk;
    case SPTRSV_OPT_MULTI_ROWS:
      if (v != 0 && v != 1 && v != 2 && v != 4) return kErrInvalidArg;
      h->mrows = static_cast<int>(v);
      return kOk;
    case SPTRSV_OPT_RESIDENCY_LIMIT:
      if (v < 0 || v > INT32_MAX) return kErrInvalidArg;
      h->res_limit = static_cast<int>(v);
      return kOk;
    case SPTRSV_OPT_BLOCK_RESIDENT:
      if (v != 0 && v != 1) return kErrInvalidArg;
      h->block_resident = static_cast<int>(v);
      return kOk;
    case SPTRSV_OPT_COOPERATIVE:
      if (v != 0 && v != 1) return kErrInvalidArg;
      h->coop = static_cast<int>(v);
      return kOk;
  }
  return kErrInvalidArg;
}

int sptrsv_get_option(sptrsv_handle_t h, sptrsv_option key, int64_t* v) {
  if (!h || !v) return kErrInvalidArg;
  switch (key) {
    case SPTRSV_OPT_ALGO: *v = h->algo; return kOk;
    case SPTRSV_OPT_GROUP: *v = h->group; return kOk;
    case SPTRSV_OPT_ENTRIES_PER_LANE: *v = h->epl; return kOk;
    case SPTRSV_OPT_SYNC: *v = h->sync; return kOk;
    case SPTRSV_OPT_SPIN_LIMIT: *v = h->spin_limit; return kOk;
    case SPTRSV_OPT_GRID: *v = h->grid; return kOk;
    case SPTRSV_OPT_TIMING: *v = h->timing; return kOk;
    case SPTRSV_OPT_WG: *v = h->wg; return kOk;
    case SPTRSV_OPT_ROWS_PER_LANE: *v = h->rpl; return kOk;
    case SPTRSV_OPT_ASSIGN: *v = h->assign; return kOk;
    case SPTRSV_OPT_POLL: *v = h->poll; return kOk;
    case SPTRSV_OPT_XP_STRIDE: *v = h->xp_stride; return kOk;
    case SPTRSV_OPT_MULTI_ROWS: *v = h->mrows; return kOk;
    case SPTRSV_OPT_RESIDENCY_LIMIT: *v = h->res_limit; return kOk;
    case SPTRSV_OPT_BLOCK_RESIDENT: *v = h->block_resident; return kOk;
    case SPTRSV_OPT_COOPERATIVE: *v = h->coop; return kOk;
  }
  return kErrInvalidArg;
}

int sptrsv_tune(sptrsv_handle_t h, const void* b, void* x, hipStream_t stream) {
  if (!h) return kErrInvalidArg;
  if (h->n == 0) return kOk;
  if (!b || !x || b == x) return kErrInvalidArg;
  if (!h->hash_valid) {
    if (const int st = ensure_pattern_host(h)) return st;
    h->hash = pattern_hash(h->n, h->rp_h.data(), h->col_h.data(), h->upper, h->unit);
    h->hash_valid = true;
  }
  {
    // a pattern tuned before in this process (same dtype and fixed algo)
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(tune_key(h));
    if (it != g_tune_cache.end()) {
      h->tuned = true;
      h->tuned_cfg = it->second;
      return kOk;
    }
  }
  // candidate schedules, restricted to the algorithm the options fix (all of
  // them under ALGO_AUTO).  Every candidate keeps the handle's lane rule (the
  // GROUP and ENTRIES_PER_LANE options), which fixes each row's summation
  // order, so all of them compute the same bits: timing noise may change
  // which one wins, never the result.  Varied: rows per lane, and for the
  // self-scheduled solve the persistent grid, chunk assignment, sync,
  // polling mode and slot width; level vs self (vs block, whose one lane per
  // row matches the rule only when every row gets one lane).
  std::vector<Config> cand;
  const int ncu = h->num_cu;
  const int grp = h->group, epl = h->epl;
  const bool self_ok = h->algo == SPTRSV_ALGO_AUTO || h->algo == SPTRSV_ALGO_SELF;
  const bool level_ok = h->algo == SPTRSV_ALGO_AUTO || h->algo == SPTRSV_ALGO_LEVEL;
  if (self_ok) {
    for (int grid : {ncu / 2, ncu, 2 * ncu, 4 * ncu})
      for (int poll : {1, 0})
        // values packed, or one per 32- or 64-byte slot (fewer per cache line
        // under concurrent stores and polls)
        for (int slot : {0, 32, 64}) {
          const int stride = slot == 0 ? 1 : slot / static_cast<int>(h->vb);
          for (int as : {SPTRSV_ASSIGN_STATIC, SPTRSV_ASSIGN_XCD}) {
            Config c{SPTRSV_ALGO_SELF, grp, epl, SPTRSV_SYNC_VALUE, 1, grid, as};
            c.poll = poll;
            c.stride = stride;
            cand.push_back(c);
          }
        }
    for (int rpl : {1, 4})
      cand.push_back({SPTRSV_ALGO_SELF, grp, epl, SPTRSV_SYNC_VALUE, rpl, ncu, SPTRSV_ASSIGN_TICKET});
    cand.push_back({SPTRSV_ALGO_SELF, grp, epl, SPTRSV_SYNC_FLAG, 1, ncu, SPTRSV_ASSIGN_TICKET});
  }
  if (level_ok)
    for (int rpl : {1, 4})
      cand.push_back({SPTRSV_ALGO_LEVEL, grp, epl, SPTRSV_SYNC_VALUE, rpl, 0, SPTRSV_ASSIGN_TICKET});
  if (h->algo == SPTRSV_ALGO_COLUMN_SELF)
    for (int grid : {ncu / 2, ncu, 2 * ncu, 4 * ncu})
      for (int as : {SPTRSV_ASSIGN_STATIC, SPTRSV_ASSIGN_XCD})
        cand.push_back({SPTRSV_ALGO_COLUMN_SELF, grp, epl, SPTRSV_SYNC_VALUE, 1, grid, as});
  if (h->algo == SPTRSV_ALGO_COLUMN_LEVEL)
    cand.push_back({SPTRSV_ALGO_COLUMN_LEVEL, grp, epl, SPTRSV_SYNC_VALUE, 1, 0, SPTRSV_ASSIGN_STATIC});
  const bool one_lane = grp == 1 || (grp == 0 && h->fwd.h.max_row_len <= epl);
  if (h->algo == SPTRSV_ALGO_BLOCK || (h->algo == SPTRSV_ALGO_AUTO && one_lane)) {
    const int st0 = build_block(h, 0, stream);
    if (st0) return st0;
    cand.push_back({SPTRSV_ALGO_BLOCK, grp, epl, SPTRSV_SYNC_VALUE, 1, 0, SPTRSV_ASSIGN_TICKET});
  }
  bool capturing = false;
  if (const int so = order_begin(h, stream, &capturing)) return so;
  if (capturing) return kErrNotSupported;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return kErrHip;
  }
  const int saved_timing = h->timing;
  h->timing = 0;
  float best = 1e30f;
  Config best_c = cand[0];
  int st = kOk;
  for (const Config& c : cand) {
    auto run = [&]() {
      return h->dtype == SPTRSV_F64 ? solve_impl<double>(h, h->fwd, c, b, x, 1, h->n, stream)
                                    : solve_impl<float>(h, h->fwd, c, b, x, 1, h->n, stream);
    };
    // level-scheduled trials cost a launch per level: skip them on very deep DAGs
    if ((c.algo == SPTRSV_ALGO_LEVEL || c.algo == SPTRSV_ALGO_COLUMN_LEVEL) &&
        h->fwd.h.nlev > 20000 && cand.size() > 1)
      continue;
    if (hipEventRecord(e0, stream) != hipSuccess) { st = kErrHip; break; }
    if ((st = run())) break;   // warm-up (also builds the chunk table)
    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      st = kErrHip;
      break;
    }
    float warm_ms = 0.f;
    (void)hipEventElapsedTime(&warm_ms, e0, e1);
    if (hipEventRecord(e0, stream) != hipSuccess) { st = kErrHip; break; }
    const int reps = warm_ms > 20.f ? 1 : 3;
    for (int r = 0; r < reps && !st; ++r) st = run();
    if (st) break;
    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      st = kErrHip;
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= reps;
    if (ms < best) {
      best = ms;
      best_c = c;
    }
  }
  h->timing = saved_timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!st) st = read_status(h, stream, true);
  const int so = order_end(h, stream, false);   // the trials used the handle's buffers
  if (st || (st = so)) return st;
  h->tuned = true;
  h->tuned_cfg = best_c;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[tune_key(h)] = best_c;
  return kOk;
}

int sptrsv_tune_multi(sptrsv_handle_t h, int32_t nrhs, int32_t ld, const void* B, void* X,
                      hipStream_t stream) {
  if (!h || nrhs < 2 || ld < h->n || ld < 1) return kErrInvalidArg;
  if (h->n == 0) return kOk;
  if (!B || !X || B == X) return kErrInvalidArg;
  // solved column by column with the single-RHS schedule: nothing to tune here
  if (multi_by_columns(h->fwd, resolve_multi(h, nrhs))) return kOk;
  const int ncu = h->num_cu;
  std::vector<Config> cand;
  const bool self_ok = h->algo == SPTRSV_ALGO_AUTO || h->algo == SPTRSV_ALGO_SELF ||
                       is_column(h->algo);
  if (self_ok)
    for (int grid : {ncu / 2, ncu, 2 * ncu, 4 * ncu, 8 * ncu})
      for (int as : {SPTRSV_ASSIGN_STATIC, SPTRSV_ASSIGN_XCD})
        for (int poll : {1, 0})
          for (int mrows : {1, 2, 4}) {
            Config c{SPTRSV_ALGO_SELF, 0, 4, SPTRSV_SYNC_VALUE, 1, grid, as};
            c.poll = poll;
            c.mrows = mrows;
            cand.push_back(c);
          }
  if (h->algo == SPTRSV_ALGO_AUTO || h->algo == SPTRSV_ALGO_LEVEL || h->algo == SPTRSV_ALGO_BLOCK ||
      cand.empty())
    cand.push_back({SPTRSV_ALGO_LEVEL, 0, 4, SPTRSV_SYNC_VALUE, 1, 0, SPTRSV_ASSIGN_TICKET});
  bool capturing = false;
  if (const int so = order_begin(h, stream, &capturing)) return so;
  if (capturing) return kErrNotSupported;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return kErrHip;
  }
  const int saved_timing = h->timing;
  h->timing = 0;
  float best = 1e30f;
  Config best_c = cand[0];
  int st = kOk;
  for (const Config& c : cand) {
    auto run = [&]() {
      return h->dtype == SPTRSV_F64 ? solve_impl<double>(h, h->fwd, c, B, X, nrhs, ld, stream)
                                    : solve_impl<float>(h, h->fwd, c, B, X, nrhs, ld, stream);
    };
    if (c.algo == SPTRSV_ALGO_LEVEL && h->fwd.h.nlev > 20000 && cand.size() > 1) continue;
    if ((st = run())) break;   // warm-up (also builds the chunk table)
    if (hipEventRecord(e0, stream) != hipSuccess) { st = kErrHip; break; }
    for (int r = 0; r < 2 && !st; ++r) st = run();
    if (st) break;
    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      st = kErrHip;
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) {
      best = ms;
      best_c = c;
    }
  }
  h->timing = saved_timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!st) st = read_status(h, stream, true);
  const int so = order_end(h, stream, false);
  if (st || (st = so)) return st;
  h->tuned_multi[nrhs] = best_c;
  return kOk;
}

int sptrsv_probe_hop(int same_xcd, int32_t iters, double* ns_per_hop) {
  if (!ns_per_hop || iters < 2) return kErrInvalidArg;
  *ns_per_hop = 0.0;
  int dev = 0, khz = 0;
  HIPCHK(hipGetDevice(&dev));
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return kErrHip;
  void* buf = nullptr;
  if (hipMalloc(&buf, 256) != hipSuccess) return kErrOom;
  int* a = static_cast<int*>(buf);
  int* b = a + 16;                       // another 64-byte line
  int* status = a + 32;
  long long* ticks = reinterpret_cast<long long*>(a + 48);
  int st = kOk;
  if (hipMemset(buf, 0, 256) != hipSuccess ||
      launch_pingpong(a, b, same_xcd ? 8 : 1, iters, 1 << 26, ticks, status, nullptr) !=
          hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    st = kErrHip;
  } else {
    int flag = 0;
    long long t = 0;
    if (hipMemcpy(&flag, status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(&t, ticks, sizeof(t), hipMemcpyDeviceToHost) != hipSuccess)
      st = kErrHip;
    else if (flag)
      st = kErrTimeout;
    else
      *ns_per_hop = static_cast<double>(t) * 1e6 / khz / (2.0 * (iters - 1));
  }
  (void)hipFree(buf);
  return st;
}

int sptrsv_get_info(sptrsv_handle_t h, int32_t* n, int64_t* nnz, int32_t* nlev, int32_t* algo,
                    int32_t* group) {
  if (!h) return kErrInvalidArg;
  const Config c = resolve(h);
  if (n) *n = h->n;
  if (nnz) *nnz = h->nnz;
  if (nlev) *nlev = h->fwd.h.nlev;
  if (algo) *algo = c.algo;
  if (group) *group = c.group;
  return kOk;
}

int sptrsv_get_schedule(sptrsv_handle_t h, int32_t* algo, int32_t* group,
                        int32_t* entries_per_lane, int32_t* sync, int32_t* rows_per_lane,
                        int32_t* grid, int32_t* assign, int32_t* poll) {
  if (!h) return kErrInvalidArg;
  const Config c = resolve(h);
  if (algo) *algo = c.algo;
  if (group) *group = c.group;
  if (entries_per_lane) *entries_per_lane = c.epl;
  if (sync) *sync = c.sync;
  if (rows_per_lane) *rows_per_lane = c.rpl;
  if (grid) *grid = c.grid;
  if (assign) *assign = c.assign;
  if (poll) *poll = c.poll;
  return kOk;
}

int sptrsv_get_xp_stride(sptrsv_handle_t h, int32_t* stride) {
  if (!h || !stride) return kErrInvalidArg;
  *stride = resolve(h).stride;
  return kOk;
}

int sptrsv_export_analysis(sptrsv_handle_t h, int transpose, int32_t* level, int32_t* ilev,
                           int32_t* jlev, int32_t* depcnt) {
  if (!h) return kErrInvalidArg;
  if (transpose) {
    const int st = build_transpose(h, h->last_stream);
    if (st) return st;
  }
  if (const int st = ensure_plan_host(transpose ? h->trn : h->fwd)) return st;
  const HostPlan& p = transpose ? h->trn.h : h->fwd.h;
  if (level) std::copy(p.level.begin(), p.level.end(), level);
  if (ilev) std::copy(p.ilev.begin(), p.ilev.end(), ilev);
  if (jlev) std::copy(p.jlev.begin(), p.jlev.end(), jlev);
  if (depcnt) std::copy(p.depcnt.begin(), p.depcnt.end(), depcnt);
  return kOk;
}

int sptrsv_get_status(sptrsv_handle_t h) {
  if (!h) return kErrInvalidArg;
  return read_status(h, h->last_stream, true);
}

int sptrsv_kernel_time(sptrsv_handle_t h, double* ms, int64_t* count, int reset) {
  if (!h) return kErrInvalidArg;
  if (const int st = fold_timing(h)) return st;
  if (ms) *ms = h->acc_ms;
  if (count) *count = h->acc_count;
  if (reset) {
    h->acc_ms = 0.0;
    h->acc_count = 0;
  }
  return kOk;
}

const char* sptrsv_status_string(int status) {
  switch (status) {
    case SPTRSV_OK: return "ok";
    case SPTRSV_ERR_INVALID_ARG: return "invalid argument";
    case SPTRSV_ERR_BAD_ROWPTR: return "row_ptr not monotone from 0 to nnz";
    case SPTRSV_ERR_BAD_COLIDX: return "column index out of range";
    case SPTRSV_ERR_NOT_TRIANGULAR: return "entry on the wrong side of the diagonal";
    case SPTRSV_ERR_DUPLICATE: return "duplicate column in a row";
    case SPTRSV_ERR_MISSING_DIAG: return "missing diagonal entry";
    case SPTRSV_ERR_ZERO_PIVOT: return "zero diagonal entry";
    case SPTRSV_ERR_HIP: return "HIP runtime error";
    case SPTRSV_ERR_OOM: return "out of memory";
    case SPTRSV_ERR_TIMEOUT: return "self-scheduled wait timed out";
    case SPTRSV_ERR_NOT_SUPPORTED: return "not supported";
    case SPTRSV_ERR_BUSY: return "handle still has live graphs";
    case SPTRSV_ERR_TOO_LARGE: return "request exceeds the fixed scratch capacity";
    case SPTRSV_ERR_NOT_RESIDENT: return "persistent grid not all resident";
  }
  return "unknown status";
}

int sptrsv_destroy(sptrsv_handle_t h) {
  if (!h) return kErrInvalidArg;
  if (h->live_graphs > 0) return kErrBusy;   // their kernels use the handle's buffers
  // the handle's own work first (hipFree also waits for the device)
  if (h->order_ev && h->order_pending) (void)hipEventSynchronize(h->order_ev);
  destroy_handle(h);
  return kOk;
}

int sptrsv_graph_capture(sptrsv_handle_t h, const void* b, void* x, int transpose,
                         hipStream_t stream, sptrsv_graph_t* out) {
  if (!h || !out || !stream) return kErrInvalidArg;
  *out = nullptr;
  if (transpose) {
    const int st = build_transpose(h, stream);
    if (st) return st;
  }
  // the work tables, occupancy figures and buffers exist before the capture
  // (their uploads are synchronous)
  if (const int st = prepare_schedule(h, transpose != 0, resolve(h), stream)) return st;
  auto* g = new (std::nothrow) sptrsv_graph_s;
  if (!g) return kErrOom;
  if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    delete g;
    return kErrHip;
  }
  const int st = solve_dispatch(h, transpose != 0, b, x, 1, h->n, stream);
  const hipError_t e = hipStreamEndCapture(stream, &g->graph);
  if (st || e != hipSuccess) {
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return st ? st : kErrHip;
  }
  if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g->graph);
    delete g;
    return kErrHip;
  }
  g->owner = h;
  g->xp_keep = h->xp_buf;
  h->live_graphs++;
  *out = g;
  return kOk;
}

int sptrsv_graph_launch(sptrsv_graph_t g, hipStream_t stream) {
  if (!g) return kErrInvalidArg;
  return hipGraphLaunch(g->exec, stream) == hipSuccess ? kOk : kErrHip;
}

int sptrsv_graph_destroy(sptrsv_graph_t g) {
  if (!g) return kErrInvalidArg;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->owner) g->owner->live_graphs--;
  delete g;   // releases the graph's hold on its position-ordered buffer
  return kOk;
}

int sptrsv_analyze_host(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                        sptrsv_uplo uplo, int unit_diag, int32_t* level, int32_t* ilev,
                        int32_t* jlev, int32_t* depcnt, int32_t* nlev) {
  if (n < 0 || nnz < 0 || !row_ptr || (nnz > 0 && !col_idx) ||
      (uplo != SPTRSV_LOWER && uplo != SPTRSV_UPPER))
    return kErrInvalidArg;
  const bool upper = uplo == SPTRSV_UPPER;
  int st = validate_pattern(n, nnz, row_ptr, col_idx, upper, unit_diag != 0, nullptr);
  if (st) return st;
  HostPlan p;
  build_plan(n, row_ptr, col_idx, nullptr, upper, unit_diag != 0, p);
  if (level) std::copy(p.level.begin(), p.level.end(), level);
  if (ilev) std::copy(p.ilev.begin(), p.ilev.end(), ilev);
  if (jlev) std::copy(p.jlev.begin(), p.jlev.end(), jlev);
  if (depcnt) std::copy(p.depcnt.begin(), p.depcnt.end(), depcnt);
  if (nlev) *nlev = p.nlev;
  return kOk;
}

}  // extern "C"
