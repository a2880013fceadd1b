// Host-side setup phase: validation, levels, level sets, layout, chunks.
// Section references are to Li, arXiv:1710.04985.
#include "analysis.hpp"

#include <algorithm>
#include <cstring>
#include <thread>

namespace sptrsv {

// Runs fn(begin, end) over [0, n) split across up to 16 host threads; the
// pieces must be independent.  Small ranges run on the calling thread.
template <typename F> static void parallel_for(int64_t n, F fn) {
  const unsigned hw = std::thread::hardware_concurrency();
  int nt = static_cast<int>(std::min<unsigned>(hw ? hw : 1, 16));
  if (n < (1 << 16) || nt <= 1) {
    fn(int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  const int64_t step = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int64_t a = t * step, b = std::min(n, a + step);
    if (a >= b) break;
    th.emplace_back([=] { fn(a, b); });
  }
  for (auto& x : th) x.join();
}

int validate_pattern(int n, int64_t nnz, const int* row_ptr, const int* col, bool upper,
                     bool unit_diag, std::vector<int>* diag_pos) {
  if (n < 0 || nnz < 0) return kErrInvalidArg;
  if (n == 0) return nnz == 0 ? kOk : kErrBadRowPtr;
  if (row_ptr[0] != 0 || row_ptr[n] != nnz) return kErrBadRowPtr;
  for (int i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return kErrBadRowPtr;
  // last_seen[j] == i marks column j as already present in row i
  std::vector<int> last_seen(n, -1);
  std::vector<int> dpos(n, -1);
  int status = kOk;
  for (int i = 0; i < n; ++i) {
    for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int j = col[k];
      if (j < 0 || j >= n) return kErrBadColIdx;
      if (upper ? (j < i) : (j > i)) status = status ? status : kErrNotTriangular;
      if (last_seen[j] == i) status = status ? status : kErrDuplicate;
      last_seen[j] = i;
      if (j == i) dpos[i] = k;
    }
  }
  if (status) return status;
  if (!unit_diag) {
    for (int i = 0; i < n; ++i)
      if (dpos[i] < 0) return kErrMissingDiag;
  }
  if (diag_pos) diag_pos->swap(dpos);
  return kOk;
}

int compute_levels(int n, const int* row_ptr, const int* col, bool upper, int* level) {
  int nlev = 0;
  for (int s = 0; s < n; ++s) {
    const int i = upper ? n - 1 - s : s;
    int lv = 0;
    for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int j = col[k];
      if (j != i) lv = std::max(lv, level[j] + 1);
    }
    level[i] = lv;
    nlev = std::max(nlev, lv + 1);
  }
  return nlev;
}

void level_sets(int n, const int* level, int nlev, int* ilev, int* jlev) {
  std::vector<int> count(nlev + 1, 0);
  for (int i = 0; i < n; ++i) count[level[i]]++;
  ilev[0] = 0;
  for (int m = 0; m < nlev; ++m) ilev[m + 1] = ilev[m] + count[m];
  std::vector<int> fill(ilev, ilev + nlev);
  for (int i = 0; i < n; ++i) jlev[fill[level[i]]++] = i;
}

void dependency_counts(int n, const int* row_ptr, const int* col, int* depcnt) {
  parallel_for(n, [&](int64_t a, int64_t b) {
    for (int i = static_cast<int>(a); i < b; ++i) {
      int c = row_ptr[i + 1] - row_ptr[i];
      for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) c -= (col[k] == i);
      depcnt[i] = c;
    }
  });
}

void transpose_pattern(int n, const int* row_ptr, const int* col, std::vector<int>& rowT,
                       std::vector<int>& colT, std::vector<int>& srcT) {
  const int64_t nnz = row_ptr[n];
  rowT.assign(n + 1, 0);
  colT.resize(nnz);
  srcT.resize(nnz);
  for (int64_t k = 0; k < nnz; ++k) rowT[col[k] + 1]++;
  for (int j = 0; j < n; ++j) rowT[j + 1] += rowT[j];
  std::vector<int> next(rowT.begin(), rowT.end() - 1);
  for (int i = 0; i < n; ++i)
    for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int d = next[col[k]]++;
      colT[d] = i;
      srcT[d] = k;
    }
}

static inline int bit_length(unsigned v) { return v ? 32 - __builtin_clz(v) : 0; }

void build_plan(int n, const int* row_ptr, const int* col, const int* src, bool upper,
                bool unit_diag, HostPlan& p) {
  p = HostPlan();
  p.n = n;
  p.upper = upper;
  p.unit_diag = unit_diag;
  p.nnz = n ? row_ptr[n] : 0;
  p.level.resize(n);
  p.jlev.resize(n);
  p.depcnt.resize(n);
  p.nlev = compute_levels(n, row_ptr, col, upper, p.level.data());
  p.ilev.resize(p.nlev + 1);
  if (n) level_sets(n, p.level.data(), p.nlev, p.ilev.data(), p.jlev.data());
  else p.ilev[0] = 0;
  dependency_counts(n, row_ptr, col, p.depcnt.data());

  // positions: inside each level, group rows by the bit length of their
  // dependency count (stable, so ascending row inside a group)
  p.pos_ilev = p.ilev;
  p.pos_row.resize(n);
  int max_len = 0;
  for (int i = 0; i < n; ++i) max_len = std::max(max_len, p.depcnt[i]);
  p.max_row_len = max_len;
  const int nclass = bit_length(static_cast<unsigned>(max_len)) + 1;
  parallel_for(p.nlev, [&](int64_t ma, int64_t mb) {
    std::vector<int> cls_count(nclass);
    for (int m = static_cast<int>(ma); m < mb; ++m) {
      const int a = p.ilev[m], b = p.ilev[m + 1];
      std::fill(cls_count.begin(), cls_count.end(), 0);
      for (int t = a; t < b; ++t) cls_count[bit_length(p.depcnt[p.jlev[t]])]++;
      int acc = a;
      for (int c = 0; c < nclass; ++c) {
        const int cnt = cls_count[c];
        cls_count[c] = acc;
        acc += cnt;
      }
      for (int t = a; t < b; ++t) {
        const int i = p.jlev[t];
        p.pos_row[cls_count[bit_length(p.depcnt[i])]++] = i;
      }
    }
  });

  // off-diagonal CSR in position order, value sources, diagonal sources
  p.off_ptr.resize(n + 1);
  p.off_ptr[0] = 0;
  for (int k = 0; k < n; ++k) p.off_ptr[k + 1] = p.off_ptr[k] + p.depcnt[p.pos_row[k]];
  p.noff = p.off_ptr[n];
  p.off_col.resize(p.noff);
  p.off_pos.resize(p.noff);
  p.off_src.resize(p.noff);
  p.diag_src.assign(n, -1);
  std::vector<int> pos_of(n);
  parallel_for(n, [&](int64_t a, int64_t b) {
    for (int k = static_cast<int>(a); k < b; ++k) pos_of[p.pos_row[k]] = k;
  });
  parallel_for(n, [&](int64_t a, int64_t b) {
    for (int k = static_cast<int>(a); k < b; ++k) {
      const int i = p.pos_row[k];
      int o = p.off_ptr[k];
      for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        const int s = src ? src[e] : e;
        if (col[e] == i) {
          if (!unit_diag) p.diag_src[k] = s;
          continue;
        }
        p.off_col[o] = col[e];
        p.off_pos[o] = pos_of[col[e]];
        p.off_src[o] = s;
        ++o;
      }
    }
  });
}

void build_push(const HostPlan& p, std::vector<int>& ptr, std::vector<int>& dst,
                std::vector<int>& src) {
  const int n = p.n;
  ptr.assign(static_cast<size_t>(n) + 1, 0);
  for (int64_t o = 0; o < p.noff; ++o) ++ptr[p.off_pos[o] + 1];
  for (int k = 0; k < n; ++k) ptr[k + 1] += ptr[k];
  dst.resize(p.noff);
  src.resize(p.noff);
  std::vector<int> fill(ptr.begin(), ptr.end() - 1);
  for (int k2 = 0; k2 < n; ++k2)
    for (int o = p.off_ptr[k2]; o < p.off_ptr[k2 + 1]; ++o) {
      const int at = fill[p.off_pos[o]]++;
      dst[at] = k2;
      src[at] = o;
    }
}

void build_chunks(const HostPlan& p, int group, int entries_per_lane, int rows_fixed,
                  int rows_per_lane, ChunkTable& t) {
  t = ChunkTable();
  if (rows_per_lane < 1) rows_per_lane = 1;
  if (rows_per_lane > kMaxRowsPerLane) rows_per_lane = kMaxRowsPerLane;
  t.level_chunk.resize(p.nlev + 1);
  if (entries_per_lane < 1) entries_per_lane = 1;
  // log2 of the lanes a row of `len` off-diagonals gets under the length rule
  auto lanes_for = [&](int len) -> int {
    int lg = 0;
    while (lg < 6 && (len + (1 << lg) - 1) / (1 << lg) > entries_per_lane) ++lg;
    return lg;
  };
  int fixed_lg = 0;
  if (group > 0) {
    while ((1 << fixed_lg) < group) ++fixed_lg;
  }
  if (rows_fixed > 0) {
    fixed_lg = 0;
    while ((64 >> fixed_lg) > rows_fixed) ++fixed_lg;
  }
  for (int m = 0; m < p.nlev; ++m) {
    t.level_chunk[m] = static_cast<int>(t.start.size());
    int k = p.pos_ilev[m];
    const int end = p.pos_ilev[m + 1];
    while (k < end) {
      int lg;
      if (rows_fixed > 0 || group > 0) lg = fixed_lg;
      else lg = lanes_for(p.off_ptr[k + 1] - p.off_ptr[k]);
      // rows_fixed: rows_per_lane rows in each of the 64 >> lg lane groups
      const int cap = rows_fixed > 0 ? (64 >> lg) * rows_per_lane
                      : lg == 0      ? 64 * rows_per_lane
                                     : 64 >> lg;
      int cnt = 1;
      while (cnt < cap && k + cnt < end) {
        if (rows_fixed <= 0 && group <= 0) {
          const int len = p.off_ptr[k + cnt + 1] - p.off_ptr[k + cnt];
          if (lanes_for(len) > lg) break;
        }
        ++cnt;
      }
      t.start.push_back(k);
      t.meta.push_back(cnt | (lg << 16));
      t.max_lg = std::max(t.max_lg, lg);
      k += cnt;
    }
  }
  t.level_chunk[p.nlev] = static_cast<int>(t.start.size());
}

void reorder_plan(const HostPlan& f, const std::vector<int>& order, HostPlan& o) {
  o = HostPlan();
  o.n = f.n;
  o.nlev = f.nlev;
  o.nnz = f.nnz;
  o.noff = f.noff;
  o.upper = f.upper;
  o.unit_diag = f.unit_diag;
  o.level = f.level;
  o.ilev = f.ilev;
  o.jlev = f.jlev;
  o.depcnt = f.depcnt;
  o.max_row_len = f.max_row_len;
  o.pos_ilev = f.pos_ilev;   // only meaningful when order keeps levels in place
  const int n = f.n;
  o.pos_row.resize(n);
  o.off_ptr.assign(n + 1, 0);
  o.diag_src.assign(n, -1);
  for (int t = 0; t < n; ++t) {
    const int k = order[t];
    o.pos_row[t] = f.pos_row[k];
    o.off_ptr[t + 1] = o.off_ptr[t] + (f.off_ptr[k + 1] - f.off_ptr[k]);
    if (f.diag_src[k] >= 0) o.diag_src[t] = static_cast<int>(f.noff) + k;
  }
  o.off_col.resize(o.noff);
  o.off_pos.resize(o.noff);
  o.off_src.resize(o.noff);
  std::vector<int> pos_of(n);
  for (int t = 0; t < n; ++t) pos_of[o.pos_row[t]] = t;
  for (int t = 0; t < n; ++t) {
    const int k = order[t];
    int d = o.off_ptr[t];
    for (int e = f.off_ptr[k]; e < f.off_ptr[k + 1]; ++e, ++d) {
      o.off_col[d] = f.off_col[e];
      o.off_pos[d] = pos_of[f.off_col[e]];
      o.off_src[d] = e;
    }
  }
}

void build_block_plan(const HostPlan& f, const std::vector<int>& seg_row0, HostPlan& out,
                      BlockInfo& info) {
  const int n = f.n;
  const int nseg = static_cast<int>(seg_row0.size()) - 1;
  std::vector<int> seg_of(n);
  for (int s = 0; s < nseg; ++s)
    for (int i = seg_row0[s]; i < seg_row0[s + 1]; ++i) seg_of[i] = s;
  // stable counting sort of f's positions by system
  std::vector<int> cnt(nseg + 1, 0);
  for (int k = 0; k < n; ++k) cnt[seg_of[f.pos_row[k]] + 1]++;
  for (int s = 0; s < nseg; ++s) cnt[s + 1] += cnt[s];
  std::vector<int> order(n);
  {
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    for (int k = 0; k < n; ++k) order[fill[seg_of[f.pos_row[k]]]++] = k;
  }
  reorder_plan(f, order, out);
  // level bounds per system (levels are consecutive runs inside a system)
  info = BlockInfo();
  info.seg_row0 = seg_row0;
  info.seg_base.assign(nseg + 1, 0);
  for (int s = 0; s < nseg; ++s) {
    const int a = cnt[s], b = cnt[s + 1];
    info.max_rows = std::max(info.max_rows, b - a);
    info.seg_base[s] = static_cast<int>(info.lev_pos.size());
    if (a == b) continue;
    int run = a;
    info.lev_pos.push_back(a);
    for (int t = a + 1; t <= b; ++t) {
      if (t == b || f.level[out.pos_row[t]] != f.level[out.pos_row[t - 1]]) {
        info.lev_pos.push_back(t);
        info.max_level = std::max(info.max_level, t - run);
        run = t;
      }
    }
  }
  info.seg_base[nseg] = static_cast<int>(info.lev_pos.size());
}

int64_t block_resident_bytes(const HostPlan& p, const BlockInfo& info, int vb) {
  int64_t best = 0;
  const int nseg = static_cast<int>(info.seg_base.size()) - 1;
  for (int s = 0; s < nseg; ++s) {
    const int lb = info.seg_base[s], nl = info.seg_base[s + 1] - lb - 1;
    if (nl <= 0) continue;
    const int q0 = info.lev_pos[lb], q1 = info.lev_pos[lb + nl];
    const int64_t ns = q1 - q0;
    const int64_t ne = static_cast<int64_t>(p.off_ptr[q1]) - p.off_ptr[q0];
    if (ns > 65535 || ne > 65535) return -1;
    const int64_t bytes = vb * (2 * ns + ne + 2) + 2 * (ns + 1) + 2 * (ne + 1) + 2 * (nl + 1);
    best = std::max(best, bytes);
  }
  return best;
}

void build_wave_lists(const ChunkTable& t, int W, int regions, std::vector<int>& ptr,
                      std::vector<int>& list, int wpb) {
  const int nch = static_cast<int>(t.start.size());
  if (wpb < 1) wpb = 1;
  if (regions < 1 || W % (regions * wpb) != 0) regions = 1;
  if (regions == 1) wpb = 1;
  const int per = W / regions;                  // wavefronts per region
  std::vector<int> owner(nch);
  std::vector<long long> taken(regions, 0);     // chunks handed out per region so far
  const int nlev = static_cast<int>(t.level_chunk.size()) - 1;
  for (int m = 0; m < nlev; ++m) {
    const int a = t.level_chunk[m], b = t.level_chunk[m + 1], L = b - a;
    for (int c = a; c < b; ++c) {
      const int r = static_cast<int>(static_cast<long long>(c - a) * regions / (L > 0 ? L : 1));
      const int k = static_cast<int>(taken[r]++ % per);   // k-th wavefront of region r
      owner[c] = (r + regions * (k / wpb)) * wpb + k % wpb;
    }
  }
  ptr.assign(W + 1, 0);
  for (int c = 0; c < nch; ++c) ptr[owner[c] + 1]++;
  for (int w = 0; w < W; ++w) ptr[w + 1] += ptr[w];
  list.resize(nch);
  std::vector<int> fill(ptr.begin(), ptr.end() - 1);
  for (int c = 0; c < nch; ++c) list[fill[owner[c]]++] = c;
}

uint64_t pattern_hash(int n, const int* row_ptr, const int* col, bool upper, bool unit_diag) {
  // 64-bit multiply / xor-shift mixing of every index (splitmix64 finaliser)
  auto mix = [](uint64_t h, uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    h ^= h >> 30;
    h *= 0xbf58476d1ce4e5b9ull;
    h ^= h >> 27;
    h *= 0x94d049bb133111ebull;
    return h ^ (h >> 31);
  };
  uint64_t h = mix(mix(mix(0x243f6a8885a308d3ull, static_cast<uint64_t>(n)), upper), unit_diag);
  if (n == 0) return h;
  const int64_t nnz = row_ptr[n];
  for (int i = 0; i <= n; ++i) h = mix(h, static_cast<uint32_t>(row_ptr[i]));
  for (int64_t k = 0; k < nnz; ++k) h = mix(h, static_cast<uint32_t>(col[k]));
  return h;
}

}  // namespace sptrsv
