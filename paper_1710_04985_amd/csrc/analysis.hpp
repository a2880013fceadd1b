// Host-side setup phase of the solver (Sec. 4.4 of Li, arXiv:1710.04985):
// pattern validation, levels (Sec. 4.1), level sets, dependency counts and
// the level-ordered layout the kernels stream.  Pure C++, no HIP calls.
#pragma once

#include <cstdint>
#include <vector>

namespace sptrsv {

// Status values match sptrsv_status in include/sptrsv.h.
enum : int {
  kOk = 0,
  kErrInvalidArg = -1,
  kErrBadRowPtr = -2,
  kErrBadColIdx = -3,
  kErrNotTriangular = -4,
  kErrDuplicate = -5,
  kErrMissingDiag = -6,
  kErrZeroPivot = -7,
  kErrHip = -8,
  kErrOom = -9,
  kErrTimeout = -10,
  kErrNotSupported = -11,
  kErrBusy = -12,
  kErrTooLarge = -13,
  kErrNotResident = -14,
};

// Checks the problem statement of Sec. 3, eq. (1) on the pattern: row_ptr
// monotone from 0 to nnz, columns in range and on the right side of the
// diagonal, no repeated column in a row, a diagonal in every row unless
// unit_diag.  diag_pos[i] receives the entry index of row i's diagonal or -1.
int validate_pattern(int n, int64_t nnz, const int* row_ptr, const int* col, bool upper,
                     bool unit_diag, std::vector<int>* diag_pos);

// Levels of Sec. 4.1, 0-based: level[i] = 0 if row i has no stored
// off-diagonal, else 1 + max level[j] over them.  Rows are visited in
// dependency order (ascending for lower, descending for upper).  Returns nlev.
int compute_levels(int n, const int* row_ptr, const int* col, bool upper, int* level);

// ilev[0..nlev] level pointers and jlev rows ordered by (level, row).
void level_sets(int n, const int* level, int nlev, int* ilev, int* jlev);

// Stored off-diagonal entries per row (the dependency counts of Sec. 4.2).
void dependency_counts(int n, const int* row_ptr, const int* col, int* depcnt);

// Pattern of T^T in CSR (the CSC of T, Sec. 3) with, for every entry of T^T,
// the index of the entry of T it came from.
void transpose_pattern(int n, const int* row_ptr, const int* col, std::vector<int>& rowT,
                       std::vector<int>& colT, std::vector<int>& srcT);

// Level-ordered layout of one triangle, as the solve kernels read it.
//   pos_row[k]  row (x index) solved at position k; positions run level by
//               level (pos_ilev), inside a level grouped by the bit length of
//               the row's off-diagonal count, ascending row inside a group.
//   off_ptr     CSR pointers of the off-diagonal entries in position order;
//   off_col     their column (x index); off_pos the position the column's
//               row is solved at; off_src their index in the caller's value
//               array (for the value gather);
//   diag_src[k] index of the diagonal value of position k, -1 for unit.
struct HostPlan {
  int n = 0;
  int nlev = 0;
  int64_t nnz = 0;                // stored entries incl. diagonal
  int64_t noff = 0;               // stored off-diagonal entries
  bool upper = false;
  bool unit_diag = false;
  std::vector<int> level, ilev, jlev, depcnt;   // canonical analysis (exported)
  std::vector<int> pos_row, pos_ilev;
  std::vector<int> off_ptr, off_col, off_pos, off_src, diag_src;
  int max_row_len = 0;            // max off-diagonal count of a row
};

// Builds the plan of the triangle (row_ptr, col); src maps an entry to its
// value index (nullptr = identity).  The pattern must have been validated.
void build_plan(int n, const int* row_ptr, const int* col, const int* src, bool upper,
                bool unit_diag, HostPlan& plan);

// Push lists of a plan (column-wise solves, Sec. 3.2): the transposition of
// the off-diagonal lists in position space.  For the column solved at
// position k, entries [ptr[k], ptr[k+1]) give the positions dst[] of the rows
// that depend on it, ascending, and src[] the index of each dependency in the
// plan's off-diagonal arrays.
void build_push(const HostPlan& plan, std::vector<int>& ptr, std::vector<int>& dst,
                std::vector<int>& src);

// Work chunks: runs of consecutive positions inside ONE level, processed by
// one 64-lane wavefront.  A chunk holds `count` rows of G = 2^lg lanes each:
// count * G <= 64 when G > 1; with G = 1 a lane may own up to rows_per_lane
// rows (count <= 64 * rows_per_lane).  Encoded as {start, count | lg << 16}.
constexpr int kMaxRowsPerLane = 4;

struct ChunkTable {
  std::vector<int> start;         // first position of each chunk
  std::vector<int> meta;          // count | (lg << 16)
  std::vector<int> level_chunk;   // chunks of level m: [level_chunk[m], level_chunk[m+1])
  int max_lg = 0;
};

// group > 0: every row gets G = group lanes (a power of two <= 64).
// group == 0: G = smallest power of two with ceil(len / G) <= entries_per_lane.
// rows_fixed > 0 overrides both: G = 64 / rows_fixed lanes per row and
// count <= rows_fixed * rows_per_lane (multi-RHS kernels, where the lanes of
// a row split right-hand sides, not entries, and each lane group may own
// rows_per_lane rows).  Otherwise rows_per_lane (1..kMaxRowsPerLane) caps the
// rows a G = 1 lane owns.
void build_chunks(const HostPlan& plan, int group, int entries_per_lane, int rows_fixed,
                  int rows_per_lane, ChunkTable& out);

// Plan whose positions are those of `f` in the order given by `order` (new
// position t holds f's position order[t]); its value sources index f's value
// buffer (off-diagonals of f, then f's diagonal).
void reorder_plan(const HostPlan& f, const std::vector<int>& order, HostPlan& out);

// Block order for independent systems (block-diagonal triangles): rows of
// system s are seg_row0[s] .. seg_row0[s+1]-1.  Positions are sorted by
// (system, level, f's order inside the level); system s has its levels'
// position bounds at lev_pos[seg_base[s] .. seg_base[s+1]-1].
struct BlockInfo {
  std::vector<int> seg_row0, seg_base, lev_pos;
  int max_rows = 0;        // rows of the largest system
  int max_level = 0;       // rows of the largest level of any system
};
void build_block_plan(const HostPlan& f, const std::vector<int>& seg_row0, HostPlan& out,
                      BlockInfo& info);

// LDS bytes the resident block kernel needs for the largest system of a block
// plan (values of vb bytes: b/x, 1/diagonal and off-diagonals; 16-bit row
// offsets, dependency positions and level bounds; one dummy entry and one
// zero slot of x for rows with fewer than four entries), or -1 if some system has
// more than 65,535 rows or off-diagonals (its local indices would not fit in
// 16 bits).  0 for a plan without rows.
int64_t block_resident_bytes(const HostPlan& p, const BlockInfo& info, int vb);

// Chunk lists of the W wavefronts of a static schedule, as CSR: wavefront w
// takes chunks list[ptr[w] .. ptr[w+1]) in that (increasing) order.  Each
// level's chunks are cut into `regions` contiguous runs; run r goes to the
// wavefronts of the workgroups b with b % regions == r (wpb wavefronts per
// workgroup; round-robin among them), so that a chunk and the chunks of
// earlier levels at the same relative place in their level land on the same
// group of workgroups (the dispatcher sends workgroup b to XCD b % 8).
// regions = 1, or W not a multiple of regions * wpb, gives the plain
// round-robin c -> c % W.
void build_wave_lists(const ChunkTable& t, int W, int regions, std::vector<int>& ptr,
                      std::vector<int>& list, int wpb = 1);

// 64-bit hash of a pattern (autotuner cache key).
uint64_t pattern_hash(int n, const int* row_ptr, const int* col, bool upper, bool unit_diag);

}  // namespace sptrsv
