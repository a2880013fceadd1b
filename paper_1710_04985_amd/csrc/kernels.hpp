// Launchers of the solve kernels (kernels.hip).  Host-callable; every
// launcher enqueues on `stream` and returns the hipError_t of the launch.
#pragma once

#include <hip/hip_runtime_api.h>
#include <cstdint>

namespace sptrsv {

// Level-ordered device copy of one triangle (see HostPlan).
struct DevPlan {
  int n = 0;
  int nlev = 0;
  int64_t noff = 0;
  int* off_ptr = nullptr;   // [n+1]
  int* off_col = nullptr;   // [noff] column (caller's row number of the dependency)
  int* off_pos = nullptr;   // [noff] position of the dependency in this plan
  int* off_src = nullptr;   // [noff]
  int* diag_src = nullptr;  // [n]
  int* pos_row = nullptr;   // [n]
  int* row_pos = nullptr;   // [n] inverse of pos_row (built on first multi-RHS solve)
  void* off_val = nullptr;  // [noff] T
  void* diag = nullptr;     // [n] T, the diagonal (source of other plans' values)
  void* dinv = nullptr;     // [n] T, 1 / diagonal (what the solves multiply by)
};

// One chunk table on the device.
struct DevChunks {
  int count = 0;
  int* start = nullptr;
  int* meta = nullptr;
  int* col = nullptr;   // column-batched tables: the right-hand side of each chunk
};

// Per-handle scratch shared by the kernels.
struct DevScratch {
  int* ticket = nullptr;     // work counter of the ticket kernels
  int* status = nullptr;     // bit 0: timeout, bit 1: zero pivot
  unsigned* epoch = nullptr; // current flag epoch (flag sync)
  unsigned* flags = nullptr; // [n] per-row ready flags (flag sync)
  int* arrive = nullptr;     // wavefronts signed in (persistent kernels' residency check)
};

enum : int { kStatusTimeout = 1, kStatusZeroPivot = 2, kStatusNotResident = 4 };

// Arguments of one solve.  The solve kernels (except flag sync and block)
// keep the solution in position order in xp: xp[k * nrhs + q] is column q of
// the row solved at position k; dependencies are read there through off_pos
// (rows of one level depend on neighbouring positions of earlier levels, so
// these gathers coalesce) and every row is also written to the caller's x.
struct SolveArgs {
  const DevPlan* plan;
  const DevChunks* chunks;
  DevScratch scratch;
  const void* b;     // caller's right-hand side(s), column stride ld
  void* x;           // caller's solution(s), column stride ld
  void* xp;          // [n * nrhs] position-ordered solution (internal)
  const void* bp = nullptr;   // several right-hand sides: [n * nrhs] position-ordered b
  int nrhs = 1;
  int ld = 0;
  int spin_limit = 1 << 22;
  int poll = 1;      // waits: 1 = two overlapped rounds over all slots, 0 = pending only
  int xp_stride = 1; // static schedules, one right-hand side: elements between xp values
  int64_t xp_col = 0;   // column-batched static solves: elements between the columns of xp
  int res_limit = 1 << 20;   // residency check: polls before a persistent grid is given up
  int coop = 0;      // persistent static grids: 1 = cooperative launch, 0 = ordinary launch
  int mrows = 1;     // static schedule, several right-hand sides: rows per lane group (1, 2, 4)
  int grid = 0;      // persistent workgroups
  int wg = 64;       // threads per workgroup
  const int* wave_ptr = nullptr;   // static schedule: per-wavefront chunk lists (CSR)
  const int* wave_list = nullptr;
};

template <typename T> hipError_t launch_gather(const DevPlan& p, const T* vals, int* status,
                                               hipStream_t s);
// xp[0 .. count) := the readiness sentinel (value sync); *arrive := 0 (the
// residency check of the persistent kernel that follows)
template <typename T> hipError_t launch_fill_sentinel(T* xp, int64_t count, int* arrive,
                                                      hipStream_t s);
// Several right-hand sides in position order: bp[k * nrhs + q] :=
// B[q * ld + pos_row[k]] (and xp := the readiness sentinel if fill), then,
// after the solve, X[q * ld + i] := xp[row_pos[i] * nrhs + q].  Tiles of 64
// rows through LDS: both sides coalesced.
template <typename T> hipError_t launch_multi_in(int n, int nrhs, int ld, const T* B,
                                                 const int* row_pos, T* bp, T* xp, bool fill,
                                                 int* arrive, hipStream_t s);
template <typename T> hipError_t launch_multi_out(int n, int nrhs, int ld, const T* xp,
                                                  const int* row_pos, T* X, hipStream_t s);
// row_pos[pos_row[k]] = k
hipError_t launch_row_pos(int n, const int* pos_row, int* row_pos, hipStream_t s);
// one launch per level for [chunk_begin, chunk_end) of one level (several
// right-hand sides: in position order, bp in, xp out)
template <typename T> hipError_t launch_level(const SolveArgs& a, int chunk_begin, int chunk_end,
                                              hipStream_t s);
// self-scheduled, value sync, chunks claimed from a ticket (any nrhs)
template <typename T> hipError_t launch_self_value(const SolveArgs& a, hipStream_t s);
// self-scheduled, flag sync, ticket (one right-hand side; reads and writes x)
// level-scheduled, one lane per row, one right-hand side: positions [k0, k1)
// of one level, a thread per row
template <typename T> hipError_t launch_level_flat(const SolveArgs& a, int k0, int k1,
                                                   hipStream_t s);
template <typename T> hipError_t launch_self_flag(const SolveArgs& a, hipStream_t s);
// self-scheduled, value sync, static round-robin chunks over an all-resident
// persistent grid (cooperative launch if a.coop), pipelined (any nrhs:
// several take k_self_multi with mrows rows per lane group)
template <typename T> hipError_t launch_self_static(const SolveArgs& a, hipStream_t s);
// one workgroup of `threads` per independent system; lds_rows > 0: x of each
// system in LDS (lds_rows >= the largest system), else in global memory
template <typename T> hipError_t launch_block(const SolveArgs& a, const int* seg_row0,
                                              const int* seg_base, const int* lev_pos, int nseg,
                                              int threads, int lds_rows, hipStream_t s);
// one workgroup of `threads` per independent system, each system's whole
// level-ordered copy in `lds_bytes` of LDS (block_resident_bytes): all
// threads copy it in and out, one wavefront walks the levels
template <typename T> hipError_t launch_block_res(const SolveArgs& a, const int* seg_base,
                                                  const int* lev_pos, int nseg, int threads,
                                                  int lds_bytes, hipStream_t s);
template <typename T> hipError_t launch_grad_vals(int n, const int* row_ptr, const int* col,
                                                  int unit_diag, const T* grad_b, const T* x,
                                                  T* grad_vals, hipStream_t s);
// flags reset (epoch wrap) and scratch initialisation
hipError_t launch_init_scratch(DevScratch sc, int n, hipStream_t s);

// occupancy of the persistent kernels: workgroups per CU at `wg` threads
template <typename T> int self_value_blocks_per_cu(int wg);
template <typename T> int self_flag_blocks_per_cu(int wg);
template <typename T> int self_static_blocks_per_cu(int wg);
template <typename T> int self_multi_blocks_per_cu(int wg, int rows);

}  // namespace sptrsv
