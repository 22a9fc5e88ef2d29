// Host-side compaction of an active set into z-runs and segments.
//
// Sec. II.A flattens the wavefunction and drops every site outside the
// region of interest.  The paper's CPU kernel notes that most sites have all
// six neighbours, with the fast-axis neighbours at +-1 and the two slow-axis
// offsets shared by consecutive sites.  Here that observation is made exact
// for whole stretches of a z-run: a run is split into segments on which each
// of the four lateral neighbours (i-1, i+1, j-1, j+1) is either absent or at
// one constant compact offset.  Kernels then need one 24-byte descriptor per
// segment instead of per-site neighbour indices.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace gpe {

enum : int32_t { SEG_RUN_BEGIN = 1, SEG_RUN_END = 2 };

struct SegHead {      // staged in LDS by the kernels
  int32_t start;      // compact index of the first site
  int32_t flags;      // SEG_RUN_BEGIN | SEG_RUN_END
};

struct SegNb {        // constant lateral offsets (0 = neighbour absent)
  int32_t xm, xp, ym, yp;
};

// The 19-point HOC stencil (App. B eq. (B2)) needs, besides the k+-1
// neighbours of the site's own run, sixteen lateral taps (di, dj, dk):
//   0-3   (-1,0,0) (1,0,0) (0,-1,0) (0,1,0)        faces
//   4-7   (-1,0,-1) (-1,0,1) (1,0,-1) (1,0,1)      xz edges
//   8-11  (0,-1,-1) (0,-1,1) (0,1,-1) (0,1,1)      yz edges
//   12-15 (-1,-1,0) (-1,1,0) (1,-1,0) (1,1,0)      xy edges
// HOC segments are stretches of a run on which every tap is absent or at one
// constant compact offset.
constexpr int HOC_TAPS = 16;
struct SegHoc {
  int32_t off[HOC_TAPS];
};
// The 27-point cubic stencil adds the eight corners (taps 16-23):
//   (-1,-1,-1) (-1,-1,1) (-1,1,-1) (-1,1,1) (1,-1,-1) (1,-1,1) (1,1,-1) (1,1,1)
constexpr int C27_TAPS = 24;
struct SegC27 {
  int32_t off[C27_TAPS];
};
extern const int8_t kHocTap[C27_TAPS][3];

struct Layout {
  int64_t n[3] = {0, 0, 0};
  double h[3] = {0, 0, 0};
  double x0[3] = {0, 0, 0};
  int64_t n_active = 0;
  // runs (merged, sorted)
  std::vector<int64_t> run_i, run_j, run_k0, run_k1, run_start;
  // segments; heads has n_segments + 1 entries, the last = {n_active, 0}
  std::vector<SegHead> heads;
  std::vector<SegNb> nbs;
  // HOC segments (built on demand by build_hoc_segments / build_c27_segments)
  std::vector<SegHead> hoc_heads;
  std::vector<SegHoc> hoc_nbs;
  std::vector<SegHead> c27_heads;
  std::vector<SegC27> c27_nbs;
  int64_t n_runs() const { return (int64_t)run_i.size(); }
  int64_t n_segments() const { return (int64_t)nbs.size(); }
};

// Fill L.hoc_heads / L.hoc_nbs, or L.c27_heads / L.c27_nbs (no-op when built).
void build_hoc_segments(Layout& L);
void build_c27_segments(Layout& L);

// Returns an empty string on success, else a description of the problem.
std::string layout_from_mask(const int64_t n[3], const uint8_t* mask, Layout& out);
std::string layout_from_runs(const int64_t n[3], int64_t nruns, const int64_t* runs, Layout& out);

}  // namespace gpe
