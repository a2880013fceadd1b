// CPU check of the library's level-ordered layout and work chunks (the
// indexing every solve kernel relies on).  Built with g++ together with the
// library's host analysis source; called from tests/test_plan_cpu.py.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "analysis.hpp"

using namespace sptrsv;

extern "C" int check_plan(int n, const int* rp, const int* col, int upper, int unit, int group,
                          int epl, int rows_fixed, int rows_per_lane) {
  HostPlan p;
  build_plan(n, rp, col, nullptr, upper != 0, unit != 0, p);
  // 1: pos_row is a permutation and every level holds the canonical rows
  std::vector<int> seen(n, 0);
  for (int k = 0; k < n; ++k) {
    if (p.pos_row[k] < 0 || p.pos_row[k] >= n || seen[p.pos_row[k]]++) return 1;
  }
  if (p.pos_ilev != p.ilev) return 2;
  for (int m = 0; m < p.nlev; ++m)
    for (int k = p.pos_ilev[m]; k < p.pos_ilev[m + 1]; ++k)
      if (p.level[p.pos_row[k]] != m) return 3;
  // 2: off-diagonal copy maps back to the caller's entries of the same row
  if (p.off_ptr[0] != 0 || p.off_ptr[n] != p.noff) return 4;
  std::vector<int> used(rp[n], 0);
  for (int k = 0; k < n; ++k) {
    const int i = p.pos_row[k];
    if (p.off_ptr[k + 1] - p.off_ptr[k] != p.depcnt[i]) return 5;
    for (int o = p.off_ptr[k]; o < p.off_ptr[k + 1]; ++o) {
      const int s = p.off_src[o];
      if (s < rp[i] || s >= rp[i + 1] || col[s] != p.off_col[o] || col[s] == i || used[s]++) return 6;
      if (upper ? p.off_col[o] <= i : p.off_col[o] >= i) return 7;
      // the dependency's position: solved at an earlier level
      const int q = p.off_pos[o];
      if (q < 0 || q >= n || p.pos_row[q] != p.off_col[o] || p.level[p.off_col[o]] >= p.level[i])
        return 17;
    }
    const int d = p.diag_src[k];
    if (unit) {
      if (d != -1) return 8;
    } else if (d < rp[i] || d >= rp[i + 1] || col[d] != i || used[d]++) {
      return 9;
    }
  }
  // 3: chunks tile the positions in order, one level each, <= 64 lanes
  ChunkTable t;
  build_chunks(p, group, epl, rows_fixed, rows_per_lane, t);
  if ((int)t.level_chunk.size() != p.nlev + 1) return 10;
  int next = 0;
  for (int m = 0; m < p.nlev; ++m) {
    for (int c = t.level_chunk[m]; c < t.level_chunk[m + 1]; ++c) {
      const int cnt = t.meta[c] & 0xffff, lg = t.meta[c] >> 16;
      // a G = 1 lane, or each lane group of a multi-RHS chunk, owns up to
      // rows_per_lane rows
      const int cap = (lg == 0 || rows_fixed > 0) ? 64 * rows_per_lane : 64;
      if (t.start[c] != next || cnt < 1 || lg < 0 || lg > 6 || (cnt << lg) > cap) return 11;
      if (rows_per_lane > kMaxRowsPerLane) return 16;
      if (t.start[c] < p.pos_ilev[m] || t.start[c] + cnt > p.pos_ilev[m + 1]) return 12;
      if (group > 0 && (1 << lg) != group) return 13;
      if (rows_fixed > 0 && (64 >> lg) != rows_fixed) return 14;
      next += cnt;
    }
  }
  if (next != n || t.level_chunk[p.nlev] != (int)t.start.size()) return 15;
  // push lists: the exact transposition of the off-diagonal lists in position
  // space, ascending dependents; their chunks tile the positions as above
  {
    std::vector<int> pptr, pdst, psrc;
    build_push(p, pptr, pdst, psrc);
    if ((int)pptr.size() != n + 1 || pptr[0] != 0 || pptr[n] != p.noff) return 21;
    std::vector<int> hit(p.noff, 0);
    for (int k = 0; k < n; ++k)
      for (int e = pptr[k]; e < pptr[k + 1]; ++e) {
        const int o = psrc[e], k2 = pdst[e];
        if (o < 0 || o >= p.noff || hit[o]++ || p.off_pos[o] != k) return 22;
        if (k2 < 0 || k2 >= n || o < p.off_ptr[k2] || o >= p.off_ptr[k2 + 1]) return 23;
        if (e > pptr[k] && pdst[e - 1] >= k2) return 24;
        if (p.level[p.pos_row[k2]] <= p.level[p.pos_row[k]]) return 25;
      }
    HostPlan view;
    view.n = n;
    view.nlev = p.nlev;
    view.pos_ilev = p.pos_ilev;
    view.off_ptr = pptr;
    ChunkTable pt;
    build_chunks(view, group, epl, 0, 1, pt);
    int nx = 0;
    for (int m = 0; m < p.nlev; ++m)
      for (int c = pt.level_chunk[m]; c < pt.level_chunk[m + 1]; ++c) {
        const int cnt = pt.meta[c] & 0xffff, lg = pt.meta[c] >> 16;
        if (pt.start[c] != nx || cnt < 1 || (cnt << lg) > 64) return 26;
        if (pt.start[c] < p.pos_ilev[m] || pt.start[c] + cnt > p.pos_ilev[m + 1]) return 27;
        nx += cnt;
      }
    if (nx != n) return 28;
  }
  // wave lists: every chunk exactly once, increasing inside each list; with
  // regions, a chunk of run r lands in a workgroup b with b % regions == r
  std::vector<int> run(t.start.size(), 0);
  for (int m = 0; m + 1 < (int)t.level_chunk.size(); ++m) {
    const int a = t.level_chunk[m], L = t.level_chunk[m + 1] - a;
    for (int c = a; c < a + L; ++c) run[c] = (int)((long long)(c - a) * 8 / (L > 0 ? L : 1));
  }
  for (int W : {1, 3, 8, 16, 64, 256}) {
    for (int regions : {1, 8}) {
      for (int wpb : {1, 2, 4}) {
        std::vector<int> ptr, list;
        build_wave_lists(t, W, regions, ptr, list, wpb);
        if ((int)ptr.size() != W + 1 || ptr[0] != 0 || ptr[W] != (int)t.start.size()) return 18;
        std::vector<int> seen(t.start.size(), 0);
        const bool split = regions == 8 && W % (8 * wpb) == 0;
        for (int w = 0; w < W; ++w)
          for (int q = ptr[w]; q < ptr[w + 1]; ++q) {
            if (list[q] < 0 || list[q] >= (int)t.start.size() || seen[list[q]]++) return 19;
            if (q > ptr[w] && list[q] <= list[q - 1]) return 20;
            if (split && (w / wpb) % 8 != run[list[q]]) return 29;
          }
      }
    }
  }
  return 0;
}

// Model of the resident block kernel (one workgroup per system, the whole
// system in LDS) on the CPU: the same byte layout, staging and level loop,
// with every LDS access bounds-checked against the size the library
// requests (block_resident_bytes).  Values are synthetic: entry e of the
// block plan weighs +-1/(e+2) or 0, b[row] = +-(row+1) or 0, 1/diagonal =
// 1/2.  With `tiny`, values and b are near 1e-200 (some b are -0) and
// 1/diagonal = 1, so x is tiny too and products underflow to signed zeros.
// The result, computed in the kernel's order (four slots per row, the
// missing ones reading the dummy of value -0), is compared bit for bit,
// signs of zeros included, with plain substitution in the block plan's order
// (a dummy of value +0 fails this).
// Returns 0, or the number of the violated check; *bytes gets the LDS size.
extern "C" int check_block_resident(int n, const int* rp, const int* col, int upper, int nseg,
                                    const int* seg_row0_in, int vb, int tiny, long long* bytes) {
  HostPlan f;
  build_plan(n, rp, col, nullptr, upper != 0, false, f);
  std::vector<int> seg_row0(seg_row0_in, seg_row0_in + nseg + 1);
  HostPlan p;
  BlockInfo info;
  build_block_plan(f, seg_row0, p, info);
  const int64_t need = block_resident_bytes(p, info, vb);
  *bytes = need;
  if (need < 0) return 0;   // not eligible: nothing to model
  // signed values with exact zeros among them, so that sums of zero occur;
  // with `tiny`, values and b near 1e-200, so that products underflow to
  // zeros of either sign, and some b are -0
  const double scale = tiny ? 1e-200 : 1.0;
  std::vector<double> b(n), x(n, 0.0), xref(n, 0.0);
  for (int i = 0; i < n; ++i)
    b[i] = i % 5 == 0 ? (tiny && i % 10 == 0 ? -0.0 : 0.0)
                      : (i & 1 ? -(i + 1.0) : i + 1.0) * scale;
  auto val = [scale](int64_t e) {
    return e % 7 == 3 ? 0.0 : (e & 1 ? -1.0 : 1.0) * scale / static_cast<double>(e + 2);
  };
  const double dinv = tiny ? 1.0 : 0.5;   // tiny: x stays near 1e-200 as well
  for (int s = 0; s < nseg; ++s) {
    const int lb = info.seg_base[s], nl = info.seg_base[s + 1] - lb - 1;
    if (nl <= 0) continue;
    const int p0 = info.lev_pos[lb], ns = info.lev_pos[lb + nl] - p0;
    const int e0 = p.off_ptr[p0], ne = p.off_ptr[p0 + ns] - e0;
    // byte layout of the kernel: T xv[ns+1], T dv[ns], T vv[ne+1], u16 rp[ns+1],
    // u16 cp[ne+1], u16 lp[nl+1]; entry ne is a dummy pointing at xv[ns] = 0
    const int64_t o_xv = 0, o_dv = o_xv + int64_t(vb) * (ns + 1), o_vv = o_dv + int64_t(vb) * ns;
    const int64_t o_rp = o_vv + int64_t(vb) * (ne + 1), o_cp = o_rp + 2 * int64_t(ns + 1);
    const int64_t o_lp = o_cp + 2 * int64_t(ne + 1), end = o_lp + 2 * int64_t(nl + 1);
    if (end > need) return 40;
    std::vector<double> xv(ns + 1), dv(ns), vv(ne + 1);
    std::vector<int> lrp(ns + 1), lcp(ne + 1), llp(nl + 1);
    for (int q = 0; q < ns; ++q) {
      const int r = p.pos_row[p0 + q];
      if (r < seg_row0[s] || r >= seg_row0[s + 1]) return 41;
      xv[q] = b[r];
      dv[q] = dinv;
      const int off = p.off_ptr[p0 + q] - e0;
      if (off < 0 || off > 65535) return 42;
      lrp[q] = off;
    }
    lrp[ns] = ne;
    xv[ns] = 0.0;
    vv[ne] = -0.0;
    lcp[ne] = ns;
    if (ns > 65535) return 49;
    for (int e = 0; e < ne; ++e) {
      vv[e] = val(e0 + e);
      const int c = p.off_pos[e0 + e] - p0;
      if (c < 0 || c >= ns || c > 65535) return 43;
      lcp[e] = c;
    }
    for (int m = 0; m <= nl; ++m) {
      const int v = info.lev_pos[lb + m] - p0;
      if (v < 0 || v > ns || v > 65535) return 44;
      llp[m] = v;
    }
    for (int q = 0; q < ns; ++q)
      if (lrp[q] > lrp[q + 1]) return 45;
    for (int m = 0; m < nl; ++m) {
      if (llp[m] >= llp[m + 1]) return 46;
      for (int q = llp[m]; q < llp[m + 1]; ++q) {
        // the kernel's order: four slots (missing entries read the dummy),
        // then the row's remaining entries
        double sum = 0.0;
        for (int u = 0; u < 4; ++u) {
          const int ec = lrp[q] + u < lrp[q + 1] ? lrp[q] + u : ne;
          if (ec < 0 || ec > ne) return 50;
          // a dependency must come from an earlier level of the same system
          if (ec < ne && lcp[ec] >= llp[m]) return 47;
          if (lcp[ec] > ns) return 51;
          sum = std::fma(vv[ec], xv[lcp[ec]], sum);
        }
        for (int e = lrp[q] + 4; e < lrp[q + 1]; ++e) {
          if (lcp[e] >= llp[m]) return 47;
          sum = std::fma(vv[e], xv[lcp[e]], sum);
        }
        xv[q] = (xv[q] - sum) * dv[q];
      }
    }
    for (int q = 0; q < ns; ++q) x[p.pos_row[p0 + q]] = xv[q];
    // plain substitution over the block plan, global indices
    for (int q = p0; q < p0 + ns; ++q) {
      double sum = 0.0;
      for (int e = p.off_ptr[q]; e < p.off_ptr[q + 1]; ++e)
        sum = std::fma(val(e), xref[p.off_col[e]], sum);
      xref[p.pos_row[q]] = (b[p.pos_row[q]] - sum) * dinv;
    }
  }
  for (int i = 0; i < n; ++i)   // bit for bit: the sign of a zero counts
    if (std::memcmp(&x[i], &xref[i], sizeof(double)) != 0) return 48;
  return 0;
}
