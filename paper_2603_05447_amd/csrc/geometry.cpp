// Host-side compaction: active set -> merged z-runs -> segments.
#include "geometry.hpp"

#include <algorithm>
#include <cstdio>
#include <limits>

namespace gpe {
namespace {

std::string check_box(const int64_t n[3]) {
  for (int d = 0; d < 3; ++d)
    if (n[d] < 1) return "geometry: every n[d] must be >= 1";
  // box linear indices must fit int64 (they are formed as (i*n1 + j)*n2 + k)
  const double prod = (double)n[0] * (double)n[1] * (double)n[2];
  if (prod > 9.0e18) return "geometry: box too large for 64-bit linear indices";
  return "";
}

struct ColumnIndex {
  // runs of column (i, j) are [first[c], first[c+1]) with c = i*n1 + j when
  // the dense column table fits; otherwise located by binary search on keys.
  const Layout* L = nullptr;
  int64_t n1 = 0;
  bool dense = false;
  std::vector<int64_t> first;
  std::vector<int64_t> keys;

  void build(const Layout& lay) {
    L = &lay;
    n1 = lay.n[1];
    const int64_t ncol = lay.n[0] * lay.n[1];
    const int64_t nr = lay.n_runs();
    dense = ncol <= (int64_t(1) << 27);
    if (dense) {
      first.assign(ncol + 1, 0);
      for (int64_t r = 0; r < nr; ++r) first[lay.run_i[r] * n1 + lay.run_j[r] + 1]++;
      for (int64_t c = 0; c < ncol; ++c) first[c + 1] += first[c];
    } else {
      keys.resize(nr);
      for (int64_t r = 0; r < nr; ++r) keys[r] = lay.run_i[r] * n1 + lay.run_j[r];
    }
  }
  void range(int64_t i, int64_t j, int64_t& b, int64_t& e) const {
    const int64_t c = i * n1 + j;
    if (dense) {
      b = first[c];
      e = first[c + 1];
    } else {
      b = std::lower_bound(keys.begin(), keys.end(), c) - keys.begin();
      e = std::upper_bound(keys.begin(), keys.end(), c) - keys.begin();
    }
  }
};

// Cut every run into stretches on which each tap (di, dj, dk) is absent or at
// one constant compact offset, and call emit(head, offsets) per stretch.
// For run q of column (i+di, j+dj) the tap of site k lies in q exactly when
// k + dk is in [k0_q, k1_q), i.e. k in [k0_q - dk, k1_q - dk), at offset
// (start_q - k0_q + dk) - (S - k0).
template <typename Emit>
void cut_runs(const Layout& L, const ColumnIndex& col, int ntaps, const int8_t (*taps)[3], Emit emit) {
  struct Piece { int64_t a, b, off; };
  std::vector<std::vector<Piece>> pieces(ntaps);
  std::vector<int64_t> cuts;
  std::vector<int32_t> off(ntaps);
  for (int64_t r = 0; r < L.n_runs(); ++r) {
    const int64_t i = L.run_i[r], j = L.run_j[r];
    const int64_t k0 = L.run_k0[r], k1 = L.run_k1[r], S = L.run_start[r];
    cuts.clear();
    cuts.push_back(k0);
    cuts.push_back(k1);
    for (int d = 0; d < ntaps; ++d) {
      pieces[d].clear();
      const int64_t ii = i + taps[d][0], jj = j + taps[d][1], dk = taps[d][2];
      if (ii < 0 || ii >= L.n[0] || jj < 0 || jj >= L.n[1]) continue;
      int64_t b, e;
      col.range(ii, jj, b, e);
      for (int64_t q = b; q < e; ++q) {
        const int64_t a = std::max(k0, L.run_k0[q] - dk);
        const int64_t z = std::min(k1, L.run_k1[q] - dk);
        if (a >= z) continue;
        pieces[d].push_back({a, z, (L.run_start[q] - L.run_k0[q] + dk) - (S - k0)});
        cuts.push_back(a);
        cuts.push_back(z);
      }
    }
    std::sort(cuts.begin(), cuts.end());
    cuts.erase(std::unique(cuts.begin(), cuts.end()), cuts.end());
    for (size_t c = 0; c + 1 < cuts.size(); ++c) {
      const int64_t a = cuts[c], z = cuts[c + 1];
      SegHead hd;
      hd.start = (int32_t)(S + (a - k0));
      hd.flags = (a == k0 ? SEG_RUN_BEGIN : 0) | (z == k1 ? SEG_RUN_END : 0);
      for (int d = 0; d < ntaps; ++d) {
        off[d] = 0;
        for (const Piece& p : pieces[d])
          if (p.a <= a && z <= p.b) { off[d] = (int32_t)p.off; break; }
      }
      emit(hd, off.data());
    }
  }
}

const int8_t kFaceTap[4][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}};

std::string build_segments(Layout& L) {
  const int64_t nr = L.n_runs();
  L.run_start.resize(nr);
  int64_t acc = 0;
  for (int64_t r = 0; r < nr; ++r) {
    L.run_start[r] = acc;
    acc += L.run_k1[r] - L.run_k0[r];
  }
  if (acc < 1) return "geometry: the active set is empty";
  if (acc > (int64_t)std::numeric_limits<int32_t>::max() - 1)
    return "geometry: more than 2^31-2 active sites";
  L.n_active = acc;

  ColumnIndex col;
  col.build(L);
  L.heads.clear();
  L.nbs.clear();
  L.heads.reserve(nr * 2 + 1);
  L.nbs.reserve(nr * 2);
  cut_runs(L, col, 4, kFaceTap, [&](const SegHead& hd, const int32_t* off) {
    L.heads.push_back(hd);
    L.nbs.push_back({off[0], off[1], off[2], off[3]});
  });
  L.heads.push_back({(int32_t)L.n_active, 0});
  return "";
}

}  // namespace

const int8_t kHocTap[C27_TAPS][3] = {
    {-1, 0, 0},   {1, 0, 0},   {0, -1, 0},  {0, 1, 0},   {-1, 0, -1}, {-1, 0, 1}, {1, 0, -1},  {1, 0, 1},
    {0, -1, -1},  {0, -1, 1},  {0, 1, -1},  {0, 1, 1},   {-1, -1, 0}, {-1, 1, 0}, {1, -1, 0},  {1, 1, 0},
    {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {-1, 1, 1},  {1, -1, -1}, {1, -1, 1}, {1, 1, -1},  {1, 1, 1}};

void build_hoc_segments(Layout& L) {
  if (!L.hoc_heads.empty()) return;
  ColumnIndex col;
  col.build(L);
  L.hoc_heads.reserve(L.heads.size() * 2);
  L.hoc_nbs.reserve(L.nbs.size() * 2);
  cut_runs(L, col, HOC_TAPS, kHocTap, [&](const SegHead& hd, const int32_t* off) {
    L.hoc_heads.push_back(hd);
    SegHoc s;
    for (int d = 0; d < HOC_TAPS; ++d) s.off[d] = off[d];
    L.hoc_nbs.push_back(s);
  });
  L.hoc_heads.push_back({(int32_t)L.n_active, 0});
}

void build_c27_segments(Layout& L) {
  if (!L.c27_heads.empty()) return;
  ColumnIndex col;
  col.build(L);
  L.c27_heads.reserve(L.heads.size() * 2);
  L.c27_nbs.reserve(L.nbs.size() * 2);
  cut_runs(L, col, C27_TAPS, kHocTap, [&](const SegHead& hd, const int32_t* off) {
    L.c27_heads.push_back(hd);
    SegC27 s;
    for (int d = 0; d < C27_TAPS; ++d) s.off[d] = off[d];
    L.c27_nbs.push_back(s);
  });
  L.c27_heads.push_back({(int32_t)L.n_active, 0});
}

std::string layout_from_runs(const int64_t n[3], int64_t nruns, const int64_t* runs, Layout& out) {
  std::string err = check_box(n);
  if (!err.empty()) return err;
  if (nruns < 1 || runs == nullptr) return "geometry: no runs given";
  Layout L;
  for (int d = 0; d < 3; ++d) L.n[d] = n[d];
  L.run_i.reserve(nruns);
  int64_t pi = -1, pj = -1, pk1 = -1;
  for (int64_t r = 0; r < nruns; ++r) {
    const int64_t i = runs[4 * r], j = runs[4 * r + 1], k0 = runs[4 * r + 2], k1 = runs[4 * r + 3];
    if (i < 0 || i >= n[0] || j < 0 || j >= n[1] || k0 < 0 || k1 > n[2] || k0 >= k1) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "geometry: run %lld = (%lld,%lld,%lld,%lld) out of the box or empty",
                    (long long)r, (long long)i, (long long)j, (long long)k0, (long long)k1);
      return buf;
    }
    const bool same_col = (i == pi && j == pj);
    if (r > 0 && (i < pi || (i == pi && j < pj) || (same_col && k0 < pk1))) {
      char buf[128];
      std::snprintf(buf, sizeof buf, "geometry: runs not sorted or overlapping at run %lld", (long long)r);
      return buf;
    }
    if (same_col && k0 == pk1) {  // touching runs form one run
      L.run_k1.back() = k1;
    } else {
      L.run_i.push_back(i);
      L.run_j.push_back(j);
      L.run_k0.push_back(k0);
      L.run_k1.push_back(k1);
    }
    pi = i; pj = j; pk1 = k1;
  }
  err = build_segments(L);
  if (!err.empty()) return err;
  out = std::move(L);
  return "";
}

std::string layout_from_mask(const int64_t n[3], const uint8_t* mask, Layout& out) {
  std::string err = check_box(n);
  if (!err.empty()) return err;
  if (mask == nullptr) return "geometry: null mask";
  Layout L;
  for (int d = 0; d < 3; ++d) L.n[d] = n[d];
  for (int64_t i = 0; i < n[0]; ++i)
    for (int64_t j = 0; j < n[1]; ++j) {
      const uint8_t* col = mask + (i * n[1] + j) * n[2];
      int64_t k = 0;
      while (k < n[2]) {
        while (k < n[2] && !col[k]) ++k;
        if (k >= n[2]) break;
        const int64_t k0 = k;
        while (k < n[2] && col[k]) ++k;
        L.run_i.push_back(i);
        L.run_j.push_back(j);
        L.run_k0.push_back(k0);
        L.run_k1.push_back(k);
      }
    }
  if (L.run_i.empty()) return "geometry: the active set is empty";
  err = build_segments(L);
  if (!err.empty()) return err;
  out = std::move(L);
  return "";
}

}  // namespace gpe
