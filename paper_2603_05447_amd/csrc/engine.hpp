// Internal interface between the C ABI layer (abi.hip) and the kernels
// (kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/gpe.h"
#include "geometry.hpp"

namespace gpe {

// One workgroup processes one chunk: a contiguous range of compact sites
// of a single instance, plus the segment descriptors overlapping it.  A chunk
// holds at most `block * spt` sites and at most MAX_CHUNK_SEGS segments (a
// chunk is cut short where a mask fragments into many short segments), so
// one lane per segment stages the chunk's segment table.
constexpr int MAX_CHUNK_SEGS = 255;
struct Chunk {
  int32_t site_begin;   // global compact index of the first site
  int32_t count;        // number of sites (<= chunk capacity)
  int32_t seg_begin;    // global index of the segment holding site_begin
  int32_t seg_count;    // segments overlapping the chunk
  int32_t inst;         // instance
  int32_t pad[3];
};

// Segment starts of one 64-site group of a chunk: group g holds the chunk's
// sites 64 g .. 64 g + 63, which one wave covers in one site slot.  A lane's
// segment is `first` plus the number of starts after the group's first site
// up to its own, so the kernels find it with a popcount instead of a search.
struct GroupSegs {
  uint64_t starts;      // bit l: the group's site l begins a segment (0 past the chunk end)
  int32_t first;        // chunk-relative segment holding the group's first site (the last one past the end)
  int32_t pad;
};

// Per-instance constants, in device memory (read by every workgroup).
struct InstParams {
  double g, dt, t0, dV;
  // T~ y = cx (y[i-1] + y[i+1]) + cy (y[j-1] + y[j+1]) + cz (y[k-1] + y[k+1]) + cd y,
  // cx = -1/(2 hx^2), ..., cd = 1/hx^2 + 1/hy^2 + 1/hz^2   (App. B, eq. (B1), hbar = m = 1)
  double cx, cy, cz, cd;
  // 19-point HOC stencil of App. B eq. (B2) as weights of T~ = -1/2 Lap:
  // faces qx, qy, qz, centre qd, edges qxy (i+-1, j+-1), qxz, qyz
  double qx, qy, qz, qd, qxy, qxz, qyz;
  double qc;            // 27-point stencil: corner weight (the q* above then hold its weights)
  double omega, norm_target;
  int32_t pot_kind, n_knots;
  int32_t chunk_begin, chunk_count;
  int64_t site_begin, n_sites;
  const void* field2;   // GPE_POT_LERP: the stage's end array (field is its start array)
  double knot_t[GPE_MAX_KNOTS];
  double knot_v[GPE_MAX_KNOTS];
};

// Per-instance results written by the finalize kernels.
struct InstOut {
  double scale;          // renormalisation factor for the next imaginary-time step
  double norm, energy, mu;
  double ov_re, ov_im;   // overlap <a|b>
  double loss;
  double fmin, fmax;     // range of the potential field
  double dmax;           // largest |psi|^2 (stability bound of the nonlinear term)
  double pad[6];
};

enum { NPART = 4 };       // partial sums per chunk

struct Plan {
  const SegHead* heads;   // segment heads (global, +1 sentinel)
  const SegNb* nbs;       // segment lateral offsets
  const Chunk* chunks;
  const InstParams* inst;
  double* partials;       // NPART x pstride, component-major: partials[r * pstride + chunk]
  double* knot_acc;       // n_chunks * GPE_MAX_KNOTS
  InstOut* out;           // n_inst
  int64_t* step;          // device step counter
  int32_t n_chunks;
  int32_t n_inst;
  int32_t xcd_map;        // chunk order mode (see chunk_index in kernels.hip)
  const int32_t* order;   // mode 4: chunk of each workgroup (n_chunks entries)
  int32_t pstride;        // stride between partial-sum components (>= n_chunks)
  int32_t off32;          // 1: every per-site array is below 4 GiB (32-bit byte offsets)
  int32_t max_seg;        // largest seg_count of any chunk (sizes the dynamic LDS)
  int32_t hoc;            // 0: 7-point stencil; 19 / 27: heads/chunks are that stencil's segments
  const SegHoc* hocnb;    // 19-point lateral taps
  const SegC27* c27nb;    // 27-point lateral taps
  const GroupSegs* groups;  // chunk_capacity / 64 per chunk, in chunk order
};

// Compiled launch variants (workgroup size x sites per lane, chunk capacity
// = product), the chunk-to-XCD order mode, and the RK4 storage scheme:
//   scheme 0: App. A form; stage 4 reads y0, y2, y3 and forms
//             -y0/3 + y2/3 + 2 y3/3 + y4/3 + dt/6 k4          (240 B/site/step in complex128)
//   scheme 1: stage 2 also writes A = (-y0 + y2 + 2 y3)/3, stage 4 reads A only
//             and forms A + y4/3 + dt/6 k4; y4 reuses y2's buffer (224 B/site/step)
//   nt: streams touched once per pass (own-site inputs, outputs) use
//       non-temporal loads and stores
//   stage: the chunk's stencil input is staged in LDS, which supplies the
//       k-1 / k+1 neighbours and the j-1 / j+1 ones inside the window; 0 loads
//       every neighbour from global memory (L1/L2 hits) and skips the barrier
struct LaunchConfig {
  int block;
  int spt;
  int xcd;
  int scheme;
  int nt;
  int stage;
};
int config_count();
LaunchConfig config_get(int i);
inline int chunk_capacity(const LaunchConfig& c) { return c.block * c.spt; }

// Kernel families (for per-kernel timing).
enum Family {
  FAM_ITP1 = 0, FAM_ITP2, FAM_RK1, FAM_RK2, FAM_RK3, FAM_RK4, FAM_OBSERVE,
  FAM_ADJ1, FAM_ADJ2, FAM_ADJ3, FAM_ADJ4, FAM_FINALIZE, FAM_POINTWISE, FAM_RKG, FAM_COPY, FAM_COUNT
};
const char* family_name(int f);

// ---- launchers (kernels.hip) -------------------------------------------
// All return hipSuccess or the launch error.  `cfg` selects the variant.
// R = double (complex128) or float (complex64).  `real`: the state is one R
// per site (real imaginary time) instead of a complex pair.
// raw_input: psi_raw already holds phi (run_itp_phi applied the diagonal
// half-step and the scale), so pass 1 applies only the Euler substep.
// scale_from_partials: the scale is formed from the norm partials of the
// previous pass 2 (which then needs no finalize), not read from the instance
template <typename R> hipError_t run_itp_pass1(const Plan& p, const LaunchConfig& cfg, const void* psi_raw,
                                               const void* prop, void* tmp, bool real, hipStream_t s,
                                               bool raw_input = false, bool scale_from_partials = false);
// phi = s psi P (1 - g |s psi|^2 dt/2) site by site (s = the instance's scale)
template <typename R> hipError_t run_itp_phi(const Plan& p, const LaunchConfig& cfg, const void* psi,
                                             const void* prop, void* phi, bool real, hipStream_t s);
template <typename R> hipError_t run_itp_pass2(const Plan& p, const LaunchConfig& cfg, const void* tmp,
                                               const void* prop, void* psi_raw, bool real, hipStream_t s);
// stage 1..4 of the memory-optimised RK4 step; Y = stencil input, y0 = step start,
// y2/y3 read by stage 4, out = output (stage 4: may equal y0).  obs: stage 1 also
// writes observation partials of y0.  `step` is the step index n (stage time
// t0 + (n + c_i) dt); step < 0 reads the device step counter instead.
template <typename R> hipError_t run_rk_stage(const Plan& p, const LaunchConfig& cfg, int stage, bool obs,
                                              const void* Y, const void* y0, const void* y2, const void* y3,
                                              const void* field, void* out, int64_t step, hipStream_t s);
// scheme-1 stages: stage 2 writes y3 = y0 + dt/2 f(Y) and A = (-y0 + Y + 2 y3)/3;
// stage 4 writes A + Y/3 + dt/6 f(Y)
template <typename R> hipError_t run_rk_stage2_fold(const Plan& p, const LaunchConfig& cfg, const void* Y,
                                                    const void* y0, const void* field, void* y3, void* A,
                                                    int64_t step, hipStream_t s);
template <typename R> hipError_t run_rk_stage4_fold(const Plan& p, const LaunchConfig& cfg, const void* Y,
                                                    const void* A, const void* field, void* out, int64_t step,
                                                    hipStream_t s);
// generic memory-optimised RK stage (App. A): out = ccur Y + sum_j hc[j] hist[j] +
// cdt f(t0 + (step + c_stage) dt, Y), hist read at the site (nh <= 5)
template <typename R> hipError_t run_rk_generic(const Plan& p, const LaunchConfig& cfg, const void* Y, double ccur,
                                                int nh, const void* const* hist, const double* hc, double cdt,
                                                double c_stage, const void* field, void* out, int64_t step,
                                                hipStream_t s);
// observation partials (|psi|^2, Re psi^H T psi, V|psi|^2, |psi|^4) of scale*psi
template <typename R> hipError_t run_observe(const Plan& p, const LaunchConfig& cfg, const void* psi,
                                             const void* field, double t_offset_steps, bool use_scale,
                                             int64_t step, hipStream_t s, bool real = false);
// adjoint stage (4..1): X = stencil input (lambda for stage 4, else u_i), Y = forward
// stage state, lam = lambda (site), lacc = running lambda, uout = next u / new lambda
template <typename R> hipError_t run_adj_stage(const Plan& p, const LaunchConfig& cfg, int stage, const void* X,
                                               const void* Y, const void* field, const void* lam, void* lacc,
                                               void* uout, int64_t step, hipStream_t s);

// pointwise helpers (chunk-parallel, one launch each)
template <typename R> hipError_t run_make_prop(const Plan& p, const LaunchConfig& cfg, const void* field,
                                               void* prop, hipStream_t s);
template <typename R> hipError_t run_apply_scale(const Plan& p, const LaunchConfig& cfg, void* psi, bool real,
                                                 hipStream_t s);
template <typename R> hipError_t run_overlap(const Plan& p, const LaunchConfig& cfg, const void* a,
                                             const void* b, hipStream_t s);
template <typename R> hipError_t run_seed_lambda(const Plan& p, const LaunchConfig& cfg, const void* target,
                                                 void* lam, hipStream_t s);
// range of a real field and (psi != nullptr) the largest |psi|^2, per instance
template <typename R> hipError_t run_field_range(const Plan& p, const LaunchConfig& cfg, const void* field,
                                                 const void* psi, hipStream_t s, bool real_psi = false);
// real = true: one R per element (potential fields) instead of a complex pair
template <typename R> hipError_t run_pack(const int64_t* run_base, const int32_t* run_start, int64_t nruns,
                                          int64_t n_active, const void* src, void* dst, bool to_box,
                                          hipStream_t s, bool real = false);
template <typename R> hipError_t run_fill_zero(void* dst, int64_t n_complex, hipStream_t s);
// z-runs of the post-selection min(va, vb) < cutoff (vb may be null) over a
// box of n0 x n1 x n2 points, column by column: with offsets == nullptr the
// number of runs of every (i, j) column goes to counts[i n1 + j]; otherwise
// the runs {i, j, k0, k1} of column c are written from row offsets[c] of runs
template <typename R> hipError_t run_column_runs(const void* va, const void* vb, int64_t n0, int64_t n1, int64_t n2,
                                                 double cutoff, int32_t* counts, const int64_t* offsets,
                                                 int64_t* runs, hipStream_t s);
// plain streaming copy of n16 16-byte elements (the achievable-bandwidth reference)
hipError_t run_stream_copy(const void* src, void* dst, size_t n16, hipStream_t s);
// destination site i <- src[iv_src[q] + i - iv_dst[q]] for its interval q, or 0 when iv_src[q] < 0
template <typename R> hipError_t run_remap(const int64_t* iv_dst, const int64_t* iv_src, int64_t n_iv,
                                           int64_t n_dst, const void* src, void* dst, hipStream_t s);

// finalize kinds
enum FinalKind { FIN_NORM_SCALE = 0, FIN_OBS = 1, FIN_OVERLAP = 2, FIN_LOSS = 3, FIN_RANGE = 4 };
hipError_t run_finalize(const Plan& p, int kind, gpe_obs* obs_dev, hipStream_t s);
hipError_t run_knot_finalize(const Plan& p, double* grads_dev /* n_inst * GPE_MAX_KNOTS */, hipStream_t s);
hipError_t run_zero_doubles(double* p, int64_t n, hipStream_t s);
hipError_t run_set_scale_one(const Plan& p, hipStream_t s);
hipError_t run_set_step(int64_t* step, int64_t value, hipStream_t s);
hipError_t run_tick(int64_t* step, int64_t delta, hipStream_t s);

// timing hooks (abi.hip): bracket a launch with events when enabled
void timing_before(int family, hipStream_t s);
void timing_after(int family, hipStream_t s);

}  // namespace gpe
