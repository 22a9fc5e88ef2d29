// HIP kernels for gfx950 (MI355X): one time step of the Gross-Pitaevskii
// equation on the compacted active sites of a masked Cartesian grid.
//
// Work decomposition.  The compact arrays (one entry per active site, box
// order with z fastest) are cut into chunks of `block * spt` consecutive
// sites; one workgroup handles one chunk.  Every pass streams its inputs
// from HBM once per site with coalesced loads:
//   * the chunk's own values plus one site on either side (the k-1 / k+1
//     neighbours along the z-runs) are staged in LDS;
//   * the segments overlapping the chunk (heads and lateral offsets) are
//     staged in LDS, and each lane finds its segment from the chunk's group
//     table: per 64 sites, the segment holding the first one and a mask of
//     the sites that begin a segment (one popcount);
//   * the lateral neighbours are taken at the segment's constant offsets:
//     j-1 / j+1 (a column away in compact order) from the staged window when
//     they fall inside it, else from global memory, and i-1 / i+1 (a plane
//     away) from global memory, where adjacent lanes read adjacent addresses
//     of planes that were (or will be) streamed as some other chunk's centre.
//     In the default chunk order each XCD (own L2) takes the same eighth of
//     every x-plane, plane after plane, so those reads hit its L2.
// The path is bandwidth bound (a 7-point stencil plus pointwise work), so
// no matrix cores are used.  Reductions (norm, energy, overlaps, knot
// gradients) accumulate in FP64 per lane, are reduced across the wavefront
// with shuffles, and written as one partial per chunk; a finalize kernel
// sums the partials of each instance in a fixed order, so results are
// bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "engine.hpp"

namespace gpe {

template <typename R> struct CT;
template <> struct CT<double> { using T = double2; };
template <> struct CT<float> { using T = float2; };

template <typename R> __device__ __forceinline__ typename CT<R>::T cmk(R a, R b) {
  typename CT<R>::T v;
  v.x = a;
  v.y = b;
  return v;
}

// native two-element vectors, for non-temporal loads and stores of (re, im)
template <typename C> struct NVec;
template <> struct NVec<double2> { typedef double T __attribute__((ext_vector_type(2))); };
template <> struct NVec<float2> { typedef float T __attribute__((ext_vector_type(2))); };

// Non-temporal (NT = true) accesses are used for streams touched once per
// pass, so that they do not displace the neighbour planes from L2.
template <bool NT, typename T> __device__ __forceinline__ T ld(const T* p) {
  if constexpr (!NT) {
    return *p;
  } else if constexpr (std::is_floating_point<T>::value) {
    return __builtin_nontemporal_load(p);
  } else {
    const auto v = __builtin_nontemporal_load(reinterpret_cast<const typename NVec<T>::T*>(p));
    T r;
    r.x = v.x;
    r.y = v.y;
    return r;
  }
}
template <bool NT, typename T> __device__ __forceinline__ void st(T* p, const T& v) {
  if constexpr (!NT) {
    *p = v;
  } else if constexpr (std::is_floating_point<T>::value) {
    __builtin_nontemporal_store(v, p);
  } else {
    typename NVec<T>::T w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<typename NVec<T>::T*>(p));
  }
}

// ---------------------------------------------------------------------------
// launch variants
// ---------------------------------------------------------------------------
// Variant 0 is the default.  Measured on the 16M-site RF bubble grid: the
// plane-eighths order (mode 4) turns the i-1 / i+1 neighbour reads into L2
// hits and beats array order by about 3 %; the contiguous-eighths order also
// removes those misses but is slower, and non-temporal single-use streams
// beat cached ones.  Every shape holds at least 256 sites per chunk (the
// grid's partial-sum scratch is sized for that).
static const LaunchConfig kConfigs[] = {
    {256, 2, 4, 1, 1, 1}, {512, 1, 0, 1, 1, 1}, {256, 1, 0, 1, 1, 1}, {256, 4, 0, 1, 1, 1}, {512, 2, 0, 1, 1, 1},
    {1024, 1, 0, 1, 1, 1}, {256, 2, 0, 1, 0, 1}, {512, 1, 0, 1, 0, 1}, {256, 2, 1, 1, 1, 1}, {256, 2, 0, 0, 1, 1},
    {256, 2, 2, 1, 1, 1}, {256, 2, 3, 1, 1, 1}, {512, 1, 2, 1, 1, 1}, {256, 2, 0, 1, 1, 1}, {512, 1, 4, 1, 1, 1},
    {256, 4, 4, 1, 1, 1}, {64, 8, 4, 1, 1, 1},   {128, 4, 4, 1, 1, 1}, {256, 8, 4, 1, 1, 1}, {256, 2, 4, 1, 1, 0},
    {256, 4, 4, 1, 1, 0},
};
int config_count() { return (int)(sizeof(kConfigs) / sizeof(kConfigs[0])); }
LaunchConfig config_get(int i) { return kConfigs[i]; }

const char* family_name(int f) {
  static const char* names[FAM_COUNT] = {"itp_pass1",  "itp_pass2",  "rk_stage1",  "rk_stage2", "rk_stage3",
                                         "rk_stage4",  "observe",    "adj_stage1", "adj_stage2", "adj_stage3",
                                         "adj_stage4", "finalize",   "pointwise",  "rk_generic", "stream_copy"};
  return (f >= 0 && f < FAM_COUNT) ? names[f] : "?";
}

// Workgroup b runs on XCD b % 8 (round-robin dispatch); each XCD has its own
// L2.  Chunk order modes:
//   0: chunk b (array order; neighbouring chunks land on different XCDs)
//   1: XCD x owns the contiguous eighth [base_x, base_x + cnt_x)
//   2, 3: blocks of 64 / 256 consecutive chunks go to one XCD, blocks dealt
//         round-robin, so neighbouring columns and planes mostly share an L2
//         while all XCDs stream from one compact region
//   4: a host-built table (Plan::order): XCD x takes the x-th eighth of the
//      chunks of every x-plane, plane after plane
__device__ __forceinline__ int chunk_index(int b, int G, int mode) {
  if (mode == 0) return b;
  const int x = b & 7, w = b >> 3;
  if (mode == 1) {
    const int q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + w;
  }
  const int B = (mode == 2) ? 64 : 256;
  const int R = G / (8 * B);          // full rounds of 8 blocks
  if (w < R * B) return (w / B) * 8 * B + x * B + (w % B);
  return b;                           // the tail keeps array order
}

// piecewise-linear Delta(t), constant outside the knots
__device__ __forceinline__ double delta_at(const InstParams& ip, double t) {
  const int n = ip.n_knots;
  if (n <= 1 || t <= ip.knot_t[0]) return ip.knot_v[0];
  if (t >= ip.knot_t[n - 1]) return ip.knot_v[n - 1];
  int k = 0;
  while (k + 2 < n && ip.knot_t[k + 1] <= t) ++k;
  return ip.knot_v[k] + (ip.knot_v[k + 1] - ip.knot_v[k]) * (t - ip.knot_t[k]) / (ip.knot_t[k + 1] - ip.knot_t[k]);
}

// fraction of the way through a stage [knot_t[0], knot_t[1]], clamped to [0, 1]
__device__ __forceinline__ double stage_lambda(const InstParams& ip, double t) {
  const double l = (t - ip.knot_t[0]) / (ip.knot_t[1] - ip.knot_t[0]);
  return l < 0.0 ? 0.0 : (l > 1.0 ? 1.0 : l);
}

// the time parameter of a potential kind: Delta(t) for RF_RAMP, the stage
// fraction for LERP, unused for STATIC
__device__ __forceinline__ double pot_param(const InstParams& ip, double t) {
  if (ip.pot_kind == GPE_POT_RF_RAMP || ip.pot_kind == GPE_POT_SHELL_RAMP) return delta_at(ip, t);
  if (ip.pot_kind == GPE_POT_LERP) return stage_lambda(ip, t);
  return 0.0;
}

// The constant of a potential kind: omega^2 for the RF-dressed form, lambda/2
// for the harmonic shell
__device__ __forceinline__ double pot_const(const InstParams& ip) {
  return ip.pot_kind == GPE_POT_SHELL_RAMP ? 0.5 * ip.omega : ip.omega * ip.omega;
}

// V at a site: u = field, u2 = second field (LERP only), p = pot_param,
// c = pot_const
template <typename R>
__device__ __forceinline__ R potential(int kind, R u, R u2, R p, R c) {
  if (kind == GPE_POT_RF_RAMP) {
    const R d = u - p;
    return sqrt(d * d + c);
  }
  if (kind == GPE_POT_SHELL_RAMP) {
    const R d = u - p;
    return c * d * d;
  }
  if (kind == GPE_POT_LERP) return (R(1) - p) * u + p * u2;
  return u;
}

// dV/dDelta of the RF-dressed potential, dV/dR0 of the harmonic shell
template <typename R>
__device__ __forceinline__ R dpot_ddelta(int kind, R u, R delta, R c) {
  if (kind == GPE_POT_RF_RAMP) {
    const R d = u - delta;
    return -d / sqrt(d * d + c);
  }
  if (kind == GPE_POT_SHELL_RAMP) return R(-2) * c * (u - delta);
  return R(0);
}

// x / 3 with the constant split into a rounded part and its exact residual
// (1 - 3 t_hi, an exact FMA, divided by 3): x t_hi + x t_lo is rounded once,
// so the stage combinations of App. A, whose coefficients of the stage states
// sum to one, carry no systematic factor 1 + (3 t_hi - 1) per step (in FP32
// t_hi = 0.33333334 is 3e-8 too large, which turned into a steady norm
// growth of 6e-8 per RK4 step).
template <typename R>
__device__ __forceinline__ R div3(R x) {
  const R hi = R(1) / R(3);
  const R lo = fma(R(-3), hi, R(1)) / R(3);
  return fma(x, hi, x * lo);
}

// c x for a coefficient c given in FP64: in FP32 the coefficient is split
// into its rounding and the remainder, so the product is rounded once
template <typename R>
__device__ __forceinline__ R mulc(double c, R x) {
  const R hi = (R)c;
  const R lo = (R)(c - (double)hi);
  return fma(x, hi, x * lo);
}

// Sum NR doubles over the workgroup; thread 0 gets the result.
template <int BLOCK, int NR>
__device__ __forceinline__ void block_sum(double (&v)[NR], double (*red)[NR]) {
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[r] += __shfl_xor(v[r], off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int r = 0; r < NR; ++r) red[wid][r] = v[r];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      double s = 0.0;
      for (int w = 0; w < BLOCK / 64; ++w) s += red[w][r];
      v[r] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// stencil passes
// ---------------------------------------------------------------------------
enum PassOp {
  OP_ITP1 = 0,   // phi = s psi P (1 - g|s psi|^2 dt/2) on load;  out = phi - dt/2 T phi
  OP_ITP2,       // chi' = chi - dt/2 T chi;  out = chi' P (1 - g|chi'|^2 dt/2);  partial |out|^2
  OP_RK1,        // out = y0 + dt/2 f(t, y0)             (Y = y0)
  OP_RK1_OBS,    // same, plus observation partials of y0
  OP_RK2,        // out = y0 + dt/2 f(t + dt/2, Y)
  OP_RK3,        // out = y0 + dt   f(t + dt/2, Y)
  OP_RK4,        // out = -y0/3 + y2/3 + 2 y3/3 + Y/3 + dt/6 f(t + dt, Y)
  OP_OBS,        // observation partials of (scale) Y
  OP_ADJ4,       // adjoint stages (see run_adj_stage)
  OP_ADJ3,
  OP_ADJ2,
  OP_ADJ1,
  OP_RK2F,       // as OP_RK2, and out2 = (-y0 + Y + 2 out)/3
  OP_RK4F,       // out = A + Y/3 + dt/6 f(t + dt, Y)    (A read through `a`)
  OP_RKG,        // generic App. A stage: out = ccur Y + sum_j hc_j h_j + cdt dt f(t + c dt, Y)
  OP_ITP1R,      // as OP_ITP1 with Y already holding phi (diagonal half-step applied by PT_PHI)
};
constexpr int RKG_MAX_HIST = 5;

template <typename R> struct PassArgs {
  using C = typename CT<R>::T;
  const C* Y;       // stencil input
  const C* a;       // RK: y0; ADJ: forward stage state; ITP: unused
  const C* b;       // RK4: y2; ADJ: lambda at the site
  const C* c;       // RK4: y3
  const R* field;   // V (static) or U (RF)
  const R* prop;    // ITP: exp(-V dt/2)
  C* out;
  C* out2;          // ADJ: running lambda (in/out)
  double c_stage;   // stage time offset in units of dt
  int64_t step;     // step index; < 0: read the device step counter (graph replay)
  int use_scale;    // OBS: multiply Y by the instance's scale
  int scale_from_partials;  // ITP1: form the scale from the norm partials of the last pass 2
  // OP_RKG: earlier stage states read at the site, their coefficients, the
  // coefficient of the stencil input itself and the k coefficient (in units of dt)
  int nh;
  const C* h[RKG_MAX_HIST];
  double hc[RKG_MAX_HIST];
  double ccur;
  double cdt;
};

// REAL: the state is real (imaginary time from a real start, Sec. II.A), one
// R per site instead of two; only the imaginary-time passes and the
// observation pass exist in that form.
// STN: the stencil.  7 is App. B eq. (B1); 19 is the higher-order compact
// stencil of eq. (B2), whose segment descriptors hold sixteen lateral taps
// (SegHoc); 27 is the cubic stencil, which adds the eight corners (SegC27).
template <typename R, int BLOCK, int SPT, int OP, bool OFF32, bool NT, bool REAL, int STN, bool STG>
__global__ __launch_bounds__(BLOCK) void k_pass(const Plan pl, const PassArgs<R> a) {
  using C = typename CT<R>::T;
  using S = typename std::conditional<REAL, R, C>::type;   // stencil state type
  constexpr bool HOC = (STN != 7);
  using D = typename std::conditional<STN == 27, SegC27,
                                      typename std::conditional<STN == 19, SegHoc, SegNb>::type>::type;
  static_assert(!REAL || OP == OP_ITP1 || OP == OP_ITP1R || OP == OP_ITP2 || OP == OP_OBS,
                "real state: ITP and OBS only");
  static_assert(STG || STN == 7, "the 19- and 27-point passes always stage");
  constexpr int CH = BLOCK * SPT;
  constexpr bool ADJ = (OP >= OP_ADJ4 && OP <= OP_ADJ1);
  constexpr bool RK = (OP >= OP_RK1 && OP <= OP_RK4) || OP == OP_RK2F || OP == OP_RK4F || OP == OP_RKG;
  constexpr bool OBSP = (OP == OP_RK1_OBS || OP == OP_OBS);
  constexpr int NR = OBSP ? 4 : ((OP == OP_ITP2 || ADJ) ? 1 : 0);
  // per-site streams read at the lane's own site
  constexpr bool NEED_A = (OP == OP_RK2 || OP == OP_RK3 || OP == OP_RK4 || ADJ || OP == OP_RK2F || OP == OP_RK4F);
  constexpr bool NEED_B = (OP == OP_RK4 || OP == OP_ADJ3 || OP == OP_ADJ2);
  constexpr bool NEED_C = (OP == OP_RK4);
  constexpr bool NEED_L = (OP == OP_ADJ3 || OP == OP_ADJ2 || OP == OP_ADJ1);
  constexpr bool NEED_F = (RK || OP == OP_OBS || ADJ);
  constexpr bool NEED_P = (OP == OP_ITP2);
  __shared__ S sy[STG ? CH + 2 : 1];
  __shared__ double red[BLOCK / 64][NR > 0 ? NR : 1];
  const S* const Yin = reinterpret_cast<const S*>(a.Y);
  S* const Yout = reinterpret_cast<S*>(a.out);
  // dynamic LDS: lateral offsets (max_seg) then segment heads (max_seg + 1)
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  D* snb = reinterpret_cast<D*>(dyn_lds);
  SegHead* sh = reinterpret_cast<SegHead*>(dyn_lds + (size_t)pl.max_seg * sizeof(D));

  const int cidx = pl.xcd_map == 4 ? pl.order[blockIdx.x] : chunk_index((int)blockIdx.x, (int)gridDim.x, pl.xcd_map);
  const Chunk ch = pl.chunks[cidx];
  const InstParams& ip = pl.inst[ch.inst];
  const int ib = (int)ip.site_begin, ie = (int)(ip.site_begin + ip.n_sites);

  const R g = (R)ip.g, dt = (R)ip.dt;
  const R cx = (R)ip.cx, cy = (R)ip.cy, cz = (R)ip.cz, cd = (R)ip.cd;
  const int kind = ip.pot_kind;
  const R omega2 = (R)pot_const(ip);
  const int64_t step = a.step >= 0 ? a.step : *pl.step;
  const double tstage = ip.t0 + ((double)step + a.c_stage) * ip.dt;
  const R delta = (R)pot_param(ip, tstage);
  const R* const field2 = reinterpret_cast<const R*>(ip.field2);
  R scale = R(1);
  if (OP == OP_ITP1 || (OP == OP_OBS && a.use_scale)) scale = (R)pl.out[ch.inst].scale;
  if constexpr (OP == OP_ITP1) {
    if (a.scale_from_partials) {
      // every workgroup sums the instance's norm partials in one fixed order
      // (the grid is small: a few partials per lane) instead of a finalize launch
      __shared__ double s_norm[BLOCK / 64];
      double v = 0.0;
      for (int c = ip.chunk_begin + (int)threadIdx.x; c < ip.chunk_begin + ip.chunk_count; c += BLOCK)
        v += pl.partials[c];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if ((threadIdx.x & 63) == 0) s_norm[threadIdx.x >> 6] = v;
      __syncthreads();
      double n = 0.0;
      for (int w = 0; w < BLOCK / 64; ++w) n += s_norm[w];
      // the same value in every lane: move it to scalar registers, where the
      // stored scale lives, so the stencil code keeps its vector registers
      const unsigned long long b = (unsigned long long)__double_as_longlong(sqrt(ip.norm_target / (ip.dV * n)));
      const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
      const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
      scale = (R)__longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    }
  }
  const R hg = g * dt * R(0.5);
  S zero;
  if constexpr (REAL) zero = R(0); else zero = cmk<R>(R(0), R(0));

  // address of element i of a per-site array; with OFF32 the byte offset is
  // formed in 32 bits (every array is below 4 GiB), giving base-register +
  // offset addressing
  auto ptr = [&](auto* base, int i) {
    using P = decltype(base);
    using T = typename std::remove_pointer<P>::type;
    if constexpr (OFF32) {
      using B = typename std::conditional<std::is_const<T>::value, const char*, char*>::type;
      return reinterpret_cast<P>(reinterpret_cast<B>(base) + (uint32_t)i * (uint32_t)sizeof(T));
    } else {
      return base + i;
    }
  };
  auto at = [&](auto* base, int i) { return ld<false>(ptr(base, i)); };       // reused stream
  auto at1 = [&](auto* base, int i) { return ld<NT>(ptr(base, i)); };         // touched once
  auto put = [&](auto* base, int i, const auto& v) { st<NT>(ptr(base, i), v); };
  // value of the stencil input at compact site s (ITP1 applies the diagonal half-step on load)
  constexpr bool diag_on_load = (OP == OP_ITP1);
  auto load = [&](int s) -> S {
    S v = at(Yin, s);
    if constexpr (REAL) {
      if (diag_on_load) {
        const R vr = v * scale;
        v = vr * (at(a.prop, s) * (R(1) - hg * vr * vr));
      } else if (OP == OP_OBS) {
        v = v * scale;
      }
    } else if (diag_on_load) {
      const R p = at(a.prop, s);
      const R vr = v.x * scale, vi = v.y * scale;
      const R f = p * (R(1) - hg * (vr * vr + vi * vi));
      v = cmk<R>(vr * f, vi * f);
    } else if (OP == OP_OBS) {
      v = cmk<R>(v.x * scale, v.y * scale);
    }
    return v;
  };

  // Load schedule.  Global loads return in issue order, and the barriers
  // below wait for LDS traffic only, so the large streams stay in flight
  // while the workgroup exchanges the small segment tables:
  //   1. segment heads / lateral offsets (small)          -> registers or LDS
  //   2. own-site streams (y0, y2, y3, A, lambda, U, P)   -> registers
  //   3. the chunk's stencil input plus one site each side -> registers
  //   registers of 1 -> LDS (waits for 1 only), barrier (LDS only): segment
  //   lookup, 4. lateral neighbour loads, registers of 3 -> LDS (waits for 2
  //   and 3 only), barrier (LDS only), arithmetic.
  constexpr int NSTG = SPT + 1;    // staging slots per lane: ceil((CH + 2) / BLOCK)
  // Segment-table slots past the end re-load the last entry (same value to
  // the same LDS slot), so these loads are unconditional and issue first.
  const SegHead* hsrc = pl.heads + ch.seg_begin;
  const D* nsrc;
  if constexpr (STN == 27) nsrc = pl.c27nb + ch.seg_begin;
  else if constexpr (STN == 19) nsrc = pl.hocnb + ch.seg_begin;
  else nsrc = pl.nbs + ch.seg_begin;
  const int t0 = threadIdx.x;
  // a chunk holds at most MAX_CHUNK_SEGS (255) segments: one slot per lane
  // covers its table for 256 lanes or more, TBL slots for fewer
  constexpr int TBL = BLOCK > MAX_CHUNK_SEGS ? 1 : (MAX_CHUNK_SEGS + BLOCK) / BLOCK;
  // The tables are held in registers and written to LDS only after the
  // streams below are issued: loads return in issue order, so that write
  // waits for the table loads alone while the streams stay in flight.  This
  // pays for the 19/27-point passes (one slot per lane, their registers are
  // free again before the lateral taps need them) and for the 7-point passes
  // in single precision and, in double, those that read one stream besides
  // their stencil input; the heavier double-precision 7-point passes
  // (measured slightly slower that way) write the tables to LDS at once.
  constexpr bool LATE_TBL = STN == 7 && (sizeof(R) == 4 || OP == OP_ITP1 || OP == OP_ITP1R || OP == OP_ITP2 ||
                                         OP == OP_RK1 || OP == OP_RK1_OBS || OP == OP_OBS);
  static_assert(sizeof(SegHead) == sizeof(int2) && sizeof(SegNb) == sizeof(int4), "table entry sizes");
  static_assert(TBL <= 4, "table slots per lane");
  // named registers (not arrays, which the compiler would keep in scratch
  // memory)
  int2 h0, h1, h2, h3;
  int4 n0, n1, n2, n3;
  auto tbl_load = [&](int q, int2& h, int4& n) {
    const int t = t0 + q * BLOCK;
    h = *reinterpret_cast<const int2*>(hsrc + min(t, ch.seg_count));
    n = *reinterpret_cast<const int4*>(nsrc + min(t, ch.seg_count - 1));
  };
  auto tbl_store = [&](int q, const int2& h, const int4& n) {
    const int t = t0 + q * BLOCK;
    *reinterpret_cast<int2*>(sh + min(t, ch.seg_count)) = h;
    *reinterpret_cast<int4*>(snb + min(t, ch.seg_count - 1)) = n;
  };
  // 19/27-point descriptors: HQ 16-byte pieces
  constexpr bool LATE_HOC = STN != 7 && TBL == 1;
  constexpr int HQ = (int)(sizeof(D) / 16);
  static_assert(!LATE_HOC || (sizeof(D) % 16 == 0 && HQ <= 6), "descriptor size");
  int4 q0, q1, q2, q3, q4, q5;
  int2 hh;
  if constexpr (LATE_HOC) {
    const int4* src4 = reinterpret_cast<const int4*>(nsrc + min(t0, ch.seg_count - 1));
    hh = *reinterpret_cast<const int2*>(hsrc + min(t0, ch.seg_count));
    q0 = src4[0];
    if constexpr (HQ > 1) q1 = src4[1];
    if constexpr (HQ > 2) q2 = src4[2];
    if constexpr (HQ > 3) q3 = src4[3];
    if constexpr (HQ > 4) q4 = src4[4];
    if constexpr (HQ > 5) q5 = src4[5];
  } else if constexpr (LATE_TBL) {
    tbl_load(0, h0, n0);
    if constexpr (TBL > 1) tbl_load(1, h1, n1);
    if constexpr (TBL > 2) tbl_load(2, h2, n2);
    if constexpr (TBL > 3) tbl_load(3, h3, n3);
  } else {
#pragma unroll
    for (int q = 0; q < TBL; ++q) {
      const int t = t0 + q * BLOCK;
      sh[min(t, ch.seg_count)] = hsrc[min(t, ch.seg_count)];
      snb[min(t, ch.seg_count - 1)] = nsrc[min(t, ch.seg_count - 1)];
    }
  }
  __builtin_amdgcn_sched_barrier(0);

  // Lanes past the end of the chunk load its last site (always valid) and
  // skip their stores.
  const int last = ch.site_begin + ch.count - 1;
  C ra[SPT], rb[SPT], rc[SPT], rl[SPT];
  R rf[SPT], rf2[SPT], rp[SPT];
#pragma unroll
  for (int m = 0; m < SPT; ++m) {
    const int sc = min(ch.site_begin + (int)threadIdx.x + m * BLOCK, last);
    if constexpr (NEED_A) ra[m] = at1(a.a, sc);
    if constexpr (NEED_B) rb[m] = at1(a.b, sc);
    if constexpr (NEED_C) rc[m] = at1(a.c, sc);
    if constexpr (NEED_L) rl[m] = at1((const C*)a.out2, sc);
    if constexpr (NEED_F) rf[m] = at1(a.field, sc);
    if constexpr (NEED_F) rf2[m] = (kind == GPE_POT_LERP) ? at1(field2, sc) : R(0);
    if constexpr (NEED_P) rp[m] = at1(a.prop, sc);
  }
  // OP_RKG: weighted sum of the earlier stage states at the lane's sites
  C rhist[SPT];
  if constexpr (OP == OP_RKG) {
#pragma unroll
    for (int m = 0; m < SPT; ++m) {
      const int sc = min(ch.site_begin + (int)threadIdx.x + m * BLOCK, last);
      R hr = R(0), hi = R(0);
#pragma unroll
      for (int j = 0; j < RKG_MAX_HIST; ++j) {
        if (j < a.nh) {
          const C v = at1(a.h[j], sc);
          hr += mulc<R>(a.hc[j], v.x);
          hi += mulc<R>(a.hc[j], v.y);
        }
      }
      rhist[m] = cmk<R>(hr, hi);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  S stg[STG ? NSTG : 1];
  // without LDS staging: the lane's own sites and their k-1 / k+1 neighbours
  // (the site itself stands in past the instance ends, where the weight is 0)
  S own[STG ? 1 : SPT], kmv[STG ? 1 : SPT], kpv[STG ? 1 : SPT];
  if constexpr (STG) {
#pragma unroll
    for (int q = 0; q < NSTG; ++q) {
      const int t = threadIdx.x + q * BLOCK;
      const int sidx = ch.site_begin - 1 + t;
      const bool in = (t < ch.count + 2) && sidx >= ib && sidx < ie;
      stg[q] = load(in ? sidx : last);
      if (!in) stg[q] = zero;
    }
  } else {
#pragma unroll
    for (int m = 0; m < SPT; ++m) {
      const int sc = min(ch.site_begin + (int)threadIdx.x + m * BLOCK, last);
      own[m] = load(sc);
      kmv[m] = load(sc > ib ? sc - 1 : sc);
      kpv[m] = load(sc + 1 < ie ? sc + 1 : sc);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (LATE_HOC) {
    int4* dst4 = reinterpret_cast<int4*>(snb + min(t0, ch.seg_count - 1));
    *reinterpret_cast<int2*>(sh + min(t0, ch.seg_count)) = hh;
    dst4[0] = q0;
    if constexpr (HQ > 1) dst4[1] = q1;
    if constexpr (HQ > 2) dst4[2] = q2;
    if constexpr (HQ > 3) dst4[3] = q3;
    if constexpr (HQ > 4) dst4[4] = q4;
    if constexpr (HQ > 5) dst4[5] = q5;
  }
  if constexpr (LATE_TBL) {
    tbl_store(0, h0, n0);
    if constexpr (TBL > 1) tbl_store(1, h1, n1);
    if constexpr (TBL > 2) tbl_store(2, h2, n2);
    if constexpr (TBL > 3) tbl_store(3, h3, n3);
  }

  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");

  // ---- segment lookup and the lateral loads of all of the lane's sites ----
  // An absent lateral neighbour (offset 0) stands for the site itself and
  // gets stencil weight 0, so there is no divergence on presence.  The j-1 /
  // j+1 neighbours lie a column away in compact order, usually inside the
  // chunk's staged window (sy[t] holds site site_begin - 1 + t for
  // t < count + 2): those are read from LDS after the staging barrier, and
  // only the rest are loaded from global memory here.  The i-1 / i+1
  // neighbours are a plane away and always loaded.
  // the lane's segment in site slot m: the group table gives the segment of
  // the wave's first site there and the segment starts after it
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const unsigned lane = threadIdx.x & 63u;
  const uint64_t upto = (2ull << lane) - 1ull;   // bits 0 .. lane
  const GroupSegs* gtab = pl.groups + (size_t)cidx * (size_t)(BLOCK * SPT / 64);
  auto seg_of = [&](int m) -> int {
    const GroupSegs gs = gtab[wave + m * (BLOCK / 64)];
    return gs.first + __popcll(gs.starts & upto & ~1ull);
  };
  const int wbase = ch.site_begin - 1;
  int js[SPT], tym[SPT], typ[SPT];
  S xm[SPT], xp[SPT], ym[SPT], yp[SPT];
  R wxm[SPT], wxp[SPT], wym[SPT], wyp[SPT];
  // HOC: value, LDS slot (-1: loaded from global) and weight of every tap.
  // An absent tap (offset 0) gets weight 0 and still loads the site itself:
  // the unconditional load is faster than a per-lane skip, whose divergent
  // loads cost more than the bytes they save
  constexpr int NT16 = STN == 27 ? C27_TAPS : (STN == 19 ? HOC_TAPS : 1);
  S hv[SPT][NT16];
  int hs[SPT][NT16];
  R hw[SPT][NT16];
  // tap weights by class: faces x, y; xz, yz, xy edges; corners
  const R cls[6] = {(R)ip.qx, (R)ip.qy, (R)ip.qxz, (R)ip.qyz, (R)ip.qxy, (R)ip.qc};
  auto tap_class = [](int t) { return t < 2 ? 0 : (t < 4 ? 1 : (t < 8 ? 2 : (t < 12 ? 3 : (t < 16 ? 4 : 5)))); };
  if constexpr (HOC) {
#pragma unroll
    for (int m = 0; m < SPT; ++m) {
      const int s = min(ch.site_begin + (int)threadIdx.x + m * BLOCK, last);
      const int j = seg_of(m);
      js[m] = j;
#pragma unroll
      for (int t = 0; t < NT16; ++t) {
        const int o = snb[j].off[t];
        // taps in the site's own x-plane (dj != 0, di == 0) are a column away
        // and usually inside the staged window
        constexpr int ytap_mask = (1 << 2) | (1 << 3) | (1 << 8) | (1 << 9) | (1 << 10) | (1 << 11);
        const int win = s - wbase + o;
        const bool lds = ((ytap_mask >> t) & 1) && win >= 0 && win < ch.count + 2;
        hs[m][t] = lds ? win : -1;
        hv[m][t] = zero;
        if (!lds) hv[m][t] = load(s + o);
        hw[m][t] = o ? cls[tap_class(t)] : R(0);
      }
    }
  } else {
#pragma unroll
  for (int m = 0; m < SPT; ++m) {
    const int s = min(ch.site_begin + (int)threadIdx.x + m * BLOCK, last);
    const int j = seg_of(m);
    js[m] = j;
    const SegNb nb = snb[j];
    xm[m] = load(s + nb.xm);
    xp[m] = load(s + nb.xp);
    const int tm = s - wbase + nb.ym, tp = s - wbase + nb.yp;
    tym[m] = (STG && tm >= 0 && tm < ch.count + 2) ? tm : -1;
    typ[m] = (STG && tp >= 0 && tp < ch.count + 2) ? tp : -1;
    ym[m] = zero;
    yp[m] = zero;
    if (tym[m] < 0) ym[m] = load(s + nb.ym);
    if (typ[m] < 0) yp[m] = load(s + nb.yp);
    wxm[m] = nb.xm ? cx : R(0);
    wxp[m] = nb.xp ? cx : R(0);
    wym[m] = nb.ym ? cy : R(0);
    wyp[m] = nb.yp ? cy : R(0);
  }
  }
  __builtin_amdgcn_sched_barrier(0);

  // the staged stencil input becomes visible to the neighbouring lanes
  if constexpr (STG) {
#pragma unroll
    for (int q = 0; q < NSTG; ++q) {
      const int t = threadIdx.x + q * BLOCK;
      if (t < CH + 2) sy[t] = stg[q];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  }

  // ---- phase B2: arithmetic and stores ----
  double acc[NR > 0 ? NR : 1];
#pragma unroll
  for (int r = 0; r < (NR > 0 ? NR : 1); ++r) acc[r] = 0.0;

#pragma unroll
  for (int m = 0; m < SPT; ++m) {
    const int l = threadIdx.x + m * BLOCK;
    if (l < ch.count) {
      const int s = ch.site_begin + l;
      const SegHead hd = sh[js[m]];
      const int send = sh[js[m] + 1].start;
      const S yc = STG ? sy[l + 1] : own[m];
      const S zm = STG ? sy[l] : kmv[m], zp = STG ? sy[l + 2] : kpv[m];
      // own-column k-1 / k+1 weight and the centre weight of the stencil
      const R wz = HOC ? (R)ip.qz : cz, wc = HOC ? (R)ip.qd : cd;
      const R wzm = (s == hd.start && (hd.flags & SEG_RUN_BEGIN)) ? R(0) : wz;
      const R wzp = (s == send - 1 && (hd.flags & SEG_RUN_END)) ? R(0) : wz;
      // sum of the weighted lateral taps (both stencils)
      R latr = R(0), lati = R(0);
      if constexpr (HOC) {
#pragma unroll
        for (int t = 0; t < NT16; ++t) {
          if (hs[m][t] >= 0) hv[m][t] = sy[hs[m][t]];
          const R wt = hw[m][t];
          if constexpr (REAL) {
            latr += wt * hv[m][t];
          } else {
            latr += wt * hv[m][t].x;
            lati += wt * hv[m][t].y;
          }
        }
      } else {
        if (tym[m] >= 0) ym[m] = sy[tym[m]];
        if (typ[m] >= 0) yp[m] = sy[typ[m]];
        if constexpr (REAL) {
          latr = wxm[m] * xm[m] + wxp[m] * xp[m] + wym[m] * ym[m] + wyp[m] * yp[m];
        } else {
          latr = wxm[m] * xm[m].x + wxp[m] * xp[m].x + wym[m] * ym[m].x + wyp[m] * yp[m].x;
          lati = wxm[m] * xm[m].y + wxp[m] * xp[m].y + wym[m] * ym[m].y + wyp[m] * yp[m].y;
        }
      }
      (void)lati;
      if constexpr (REAL) {
        // T~ y at s, real state
        const R lt = latr + wzm * zm + wzp * zp + wc * yc;
        if constexpr (OP == OP_ITP1 || OP == OP_ITP1R) {
          put(Yout, s, yc - R(0.5) * dt * lt);
        } else if constexpr (OP == OP_ITP2) {
          const R q = yc - R(0.5) * dt * lt;
          const R w = q * (rp[m] * (R(1) - hg * q * q));
          put(Yout, s, w);
          acc[0] += (double)w * (double)w;
        } else {
          const R V = potential<R>(kind, rf[m], rf2[m], delta, omega2);
          const double d = (double)yc * (double)yc;
          acc[0] += d;
          acc[1] += (double)yc * (double)lt;
          acc[2] += (double)V * d;
          acc[3] += d * d;
        }
      } else {
      // T~ y at s
      const R lr = latr + wzm * zm.x + wzp * zp.x + wc * yc.x;
      const R li = lati + wzm * zm.y + wzp * zp.y + wc * yc.y;

      if constexpr (OP == OP_ITP1 || OP == OP_ITP1R) {
        put(a.out, s, cmk<R>(yc.x - R(0.5) * dt * lr, yc.y - R(0.5) * dt * li));
      } else if constexpr (OP == OP_ITP2) {
        const R qr = yc.x - R(0.5) * dt * lr, qi = yc.y - R(0.5) * dt * li;
        const R f = rp[m] * (R(1) - hg * (qr * qr + qi * qi));
        const R wr = qr * f, wi = qi * f;
        put(a.out, s, cmk<R>(wr, wi));
        acc[0] += (double)wr * (double)wr + (double)wi * (double)wi;
      } else if constexpr (OP == OP_OBS) {
        const R V = potential<R>(kind, rf[m], rf2[m], delta, omega2);
        const double d = (double)yc.x * (double)yc.x + (double)yc.y * (double)yc.y;
        acc[0] += d;
        acc[1] += (double)yc.x * (double)lr + (double)yc.y * (double)li;
        acc[2] += (double)V * d;
        acc[3] += d * d;
      } else if constexpr (RK) {
        const R V = potential<R>(kind, rf[m], rf2[m], delta, omega2);
        const R dens = yc.x * yc.x + yc.y * yc.y;
        const R w = V + g * dens;
        const R hr = lr + w * yc.x, hi = li + w * yc.y;   // H y
        const R fr = hi, fi = -hr;                         // f = -i H y
        if constexpr (OP == OP_RK1 || OP == OP_RK1_OBS) {
          put(a.out, s, cmk<R>(yc.x + R(0.5) * dt * fr, yc.y + R(0.5) * dt * fi));
          if constexpr (OP == OP_RK1_OBS) {
            const double d = (double)dens;
            acc[0] += d;
            acc[1] += (double)yc.x * (double)lr + (double)yc.y * (double)li;
            acc[2] += (double)V * d;
            acc[3] += d * d;
          }
        } else if constexpr (OP == OP_RK2 || OP == OP_RK3) {
          const C y0 = ra[m];
          const R cc = (OP == OP_RK2) ? R(0.5) * dt : dt;
          put(a.out, s, cmk<R>(y0.x + cc * fr, y0.y + cc * fi));
        } else if constexpr (OP == OP_RK2F) {
          const C y0 = ra[m];
          const R y3r = y0.x + R(0.5) * dt * fr, y3i = y0.y + R(0.5) * dt * fi;
          put(a.out, s, cmk<R>(y3r, y3i));
          put(a.out2, s, cmk<R>(div3<R>((yc.x - y0.x) + R(2) * y3r), div3<R>((yc.y - y0.y) + R(2) * y3i)));
        } else if constexpr (OP == OP_RK4F) {
          const C A = ra[m];
          const R c6 = dt / R(6);
          put(a.out, s, cmk<R>(A.x + div3<R>(yc.x) + c6 * fr, A.y + div3<R>(yc.y) + c6 * fi));
        } else if constexpr (OP == OP_RKG) {
          const R cdt = (R)a.cdt * dt;
          put(a.out, s, cmk<R>(rhist[m].x + mulc<R>(a.ccur, yc.x) + cdt * fr,
                               rhist[m].y + mulc<R>(a.ccur, yc.y) + cdt * fi));
        } else {
          const C y0 = ra[m], y2 = rb[m], y3 = rc[m];
          const R c6 = dt / R(6);
          const R orr = div3<R>((y2.x - y0.x) + yc.x + R(2) * y3.x) + c6 * fr;
          const R oi = div3<R>((y2.y - y0.y) + yc.y + R(2) * y3.y) + c6 * fi;
          put(a.out, s, cmk<R>(orr, oi));
        }
      } else if constexpr (ADJ) {
        // u = f X, T u = f T X  (stage 4: X = lambda, f = b_4 = 1/6)
        const R ur = (OP == OP_ADJ4) ? R(0.5) * div3<R>(yc.x) : yc.x;
        const R ui = (OP == OP_ADJ4) ? R(0.5) * div3<R>(yc.y) : yc.y;
        const R tur = (OP == OP_ADJ4) ? R(0.5) * div3<R>(lr) : lr;
        const R tui = (OP == OP_ADJ4) ? R(0.5) * div3<R>(li) : li;
        const C Y = ra[m];
        const R u0 = rf[m];
        const R V = potential<R>(kind, u0, R(0), delta, omega2);
        const R dVd = dpot_ddelta<R>(kind, u0, delta, omega2);
        const R d2 = Y.x * Y.x + Y.y * Y.y;
        const R w = V + R(2) * g * d2;
        // A = T u + (V + 2 g |Y|^2) u ;  B = g Y^2 conj(u)
        const R Ar = tur + w * ur, Ai = tui + w * ui;
        const R y2r = Y.x * Y.x - Y.y * Y.y, y2i = R(2) * Y.x * Y.y;
        const R Br = g * (y2r * ur + y2i * ui), Bi = g * (y2i * ur - y2r * ui);
        // theta = dt i (A - B)
        const R thr = -dt * (Ai - Bi), thi = dt * (Ar - Br);
        acc[0] += (double)dVd * ((double)ur * (double)Y.y - (double)ui * (double)Y.x);
        if constexpr (OP == OP_ADJ4) {
          // lambda = X;  u_3 = lambda/3 + theta_4;  running lambda = lambda + theta_4
          put(a.out, s, cmk<R>(div3<R>(yc.x) + thr, div3<R>(yc.y) + thi));
          put(a.out2, s, cmk<R>(yc.x + thr, yc.y + thi));
        } else if constexpr (OP == OP_ADJ3 || OP == OP_ADJ2) {
          const C lam = rb[m];
          const C lacc = rl[m];
          // b_3 = 1/3, b_2 = 1/6
          const R bf = (OP == OP_ADJ3) ? R(1) : R(0.5);
          put(a.out, s, cmk<R>(bf * div3<R>(lam.x) + R(0.5) * thr, bf * div3<R>(lam.y) + R(0.5) * thi));
          put(a.out2, s, cmk<R>(lacc.x + thr, lacc.y + thi));
        } else {
          const C lacc = rl[m];
          put(a.out, s, cmk<R>(lacc.x + thr, lacc.y + thi));
        }
      }
      }  // complex state
    }
  }

  if constexpr (NR > 0) {
    block_sum<BLOCK, (NR > 0 ? NR : 1)>(acc, red);
    if (threadIdx.x == 0) {
      if constexpr (ADJ) {
        // dL/dDelta_k += dt * phi_k(t_i) * q  (hat functions of the ramp knots)
        if (kind == GPE_POT_RF_RAMP || kind == GPE_POT_SHELL_RAMP) {
          const int n = ip.n_knots;
          const double q = ip.dt * acc[0];
          double* ka = pl.knot_acc + (size_t)cidx * GPE_MAX_KNOTS;
          if (n <= 1 || tstage <= ip.knot_t[0]) {
            ka[0] += q;
          } else if (tstage >= ip.knot_t[n - 1]) {
            ka[n - 1] += q;
          } else {
            int k = 0;
            while (k + 2 < n && ip.knot_t[k + 1] <= tstage) ++k;
            const double lam = (tstage - ip.knot_t[k]) / (ip.knot_t[k + 1] - ip.knot_t[k]);
            ka[k] += (1.0 - lam) * q;
            ka[k + 1] += lam * q;
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) pl.partials[(size_t)r * pl.pstride + cidx] = acc[r];
      }
    }
  }
}

// Shapes of 256 or more lanes and up to 4 sites per lane are compiled with and
// without non-temporal streams; the smaller workgroups and 8 sites per lane
// only with them, and the variant without LDS staging for 256 x 2 and 256 x 4.
template <int BLOCK, int SPT, typename R, int OP, bool REAL>
static hipError_t launch_pass(const Plan& p, const LaunchConfig& cfg, const PassArgs<R>& a, hipStream_t s) {
  constexpr bool BOTH_NT = BLOCK >= 256 && SPT <= 4;
  constexpr bool NO_STAGE = BLOCK == 256 && (SPT == 2 || SPT == 4);
  const size_t dyn = (size_t)p.max_seg * sizeof(SegNb) + (size_t)(p.max_seg + 1) * sizeof(SegHead);
  if (!p.off32) {
    hipLaunchKernelGGL((k_pass<R, 256, 2, OP, false, false, REAL, 7, true>), dim3(p.n_chunks), dim3(256), dyn, s, p,
                       a);
  } else if (!cfg.stage) {
    if constexpr (NO_STAGE) {
      if (!cfg.nt) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_pass<R, BLOCK, SPT, OP, true, true, REAL, 7, false>), dim3(p.n_chunks), dim3(BLOCK), dyn,
                         s, p, a);
    } else {
      return hipErrorInvalidValue;
    }
  } else if (cfg.nt) {
    hipLaunchKernelGGL((k_pass<R, BLOCK, SPT, OP, true, true, REAL, 7, true>), dim3(p.n_chunks), dim3(BLOCK), dyn, s,
                       p, a);
  } else {
    if constexpr (BOTH_NT)
      hipLaunchKernelGGL((k_pass<R, BLOCK, SPT, OP, true, false, REAL, 7, true>), dim3(p.n_chunks), dim3(BLOCK), dyn,
                         s, p, a);
    else
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The 19- and 27-point stencils hold 16 / 24 lateral values per site in
// registers, so they are compiled for one site per lane and 32-bit offsets only.
template <typename R, int OP, bool REAL, int STN>
static hipError_t launch_pass_hoc(const Plan& p, const LaunchConfig& cfg, const PassArgs<R>& a, hipStream_t s) {
  using D = typename std::conditional<STN == 27, SegC27, SegHoc>::type;
  if (!p.off32 || cfg.block != 256 || cfg.spt != 1) return hipErrorInvalidValue;
  const size_t dyn = (size_t)p.max_seg * sizeof(D) + (size_t)(p.max_seg + 1) * sizeof(SegHead);
  if (cfg.nt)
    hipLaunchKernelGGL((k_pass<R, 256, 1, OP, true, true, REAL, STN, true>), dim3(p.n_chunks), dim3(256), dyn, s, p,
                       a);
  else
    hipLaunchKernelGGL((k_pass<R, 256, 1, OP, true, false, REAL, STN, true>), dim3(p.n_chunks), dim3(256), dyn, s, p,
                       a);
  return hipGetLastError();
}

template <typename R, int OP, bool REAL = false>
static hipError_t dispatch_pass(const Plan& p, const LaunchConfig& cfg, const PassArgs<R>& a, hipStream_t s) {
  if (p.n_chunks <= 0) return hipSuccess;
  if (p.hoc == 19) return launch_pass_hoc<R, OP, REAL, 19>(p, cfg, a, s);
  if (p.hoc == 27) return launch_pass_hoc<R, OP, REAL, 27>(p, cfg, a, s);
  // arrays of 4 GiB or more use 64-bit addressing with the 256 x 2 shape (the
  // chunk table of a grid that large is built for that shape)
  if (cfg.block == 256 && cfg.spt == 1) return launch_pass<256, 1, R, OP, REAL>(p, cfg, a, s);
  if (cfg.block == 256 && cfg.spt == 2) return launch_pass<256, 2, R, OP, REAL>(p, cfg, a, s);
  if (cfg.block == 256 && cfg.spt == 4) return launch_pass<256, 4, R, OP, REAL>(p, cfg, a, s);
  if (cfg.block == 512 && cfg.spt == 1) return launch_pass<512, 1, R, OP, REAL>(p, cfg, a, s);
  if (cfg.block == 512 && cfg.spt == 2) return launch_pass<512, 2, R, OP, REAL>(p, cfg, a, s);
  if (cfg.block == 1024 && cfg.spt == 1) return launch_pass<1024, 1, R, OP, REAL>(p, cfg, a, s);
  if (cfg.block == 256 && cfg.spt == 8) return launch_pass<256, 8, R, OP, REAL>(p, cfg, a, s);
  if (cfg.block == 128 && cfg.spt == 4) return launch_pass<128, 4, R, OP, REAL>(p, cfg, a, s);
  if (cfg.block == 64 && cfg.spt == 8) return launch_pass<64, 8, R, OP, REAL>(p, cfg, a, s);
  return hipErrorInvalidValue;
}

template <typename R>
static PassArgs<R> pass_args() {
  PassArgs<R> a;
  a.Y = a.a = a.b = a.c = nullptr;
  a.field = a.prop = nullptr;
  a.out = a.out2 = nullptr;
  a.c_stage = 0.0;
  a.step = -1;
  a.use_scale = 0;
  a.scale_from_partials = 0;
  a.nh = 0;
  for (int j = 0; j < RKG_MAX_HIST; ++j) {
    a.h[j] = nullptr;
    a.hc[j] = 0.0;
  }
  a.ccur = 0.0;
  a.cdt = 0.0;
  return a;
}

template <typename R>
hipError_t run_itp_pass1(const Plan& p, const LaunchConfig& cfg, const void* psi_raw, const void* prop, void* tmp,
                         bool real, hipStream_t s, bool raw_input, bool scale_from_partials) {
  using C = typename CT<R>::T;
  PassArgs<R> a = pass_args<R>();
  a.scale_from_partials = scale_from_partials ? 1 : 0;
  a.Y = (const C*)psi_raw;
  a.prop = (const R*)prop;
  a.out = (C*)tmp;
  timing_before(FAM_ITP1, s);
  hipError_t e;
  if (raw_input)
    e = real ? dispatch_pass<R, OP_ITP1R, true>(p, cfg, a, s) : dispatch_pass<R, OP_ITP1R>(p, cfg, a, s);
  else
    e = real ? dispatch_pass<R, OP_ITP1, true>(p, cfg, a, s) : dispatch_pass<R, OP_ITP1>(p, cfg, a, s);
  timing_after(FAM_ITP1, s);
  return e;
}

template <typename R>
hipError_t run_itp_pass2(const Plan& p, const LaunchConfig& cfg, const void* tmp, const void* prop, void* psi_raw,
                         bool real, hipStream_t s) {
  using C = typename CT<R>::T;
  PassArgs<R> a = pass_args<R>();
  a.Y = (const C*)tmp;
  a.prop = (const R*)prop;
  a.out = (C*)psi_raw;
  timing_before(FAM_ITP2, s);
  hipError_t e = real ? dispatch_pass<R, OP_ITP2, true>(p, cfg, a, s) : dispatch_pass<R, OP_ITP2>(p, cfg, a, s);
  timing_after(FAM_ITP2, s);
  return e;
}

template <typename R>
hipError_t run_rk_stage(const Plan& p, const LaunchConfig& cfg, int stage, bool obs, const void* Y, const void* y0,
                        const void* y2, const void* y3, const void* field, void* out, int64_t step, hipStream_t s) {
  using C = typename CT<R>::T;
  PassArgs<R> a = pass_args<R>();
  a.Y = (const C*)Y;
  a.a = (const C*)y0;
  a.b = (const C*)y2;
  a.c = (const C*)y3;
  a.field = (const R*)field;
  a.out = (C*)out;
  static const double cst[4] = {0.0, 0.5, 0.5, 1.0};
  if (stage < 1 || stage > 4) return hipErrorInvalidValue;
  a.c_stage = cst[stage - 1];
  a.step = step;
  const int fam = FAM_RK1 + stage - 1;
  timing_before(fam, s);
  hipError_t e;
  switch (stage) {
    case 1: e = obs ? dispatch_pass<R, OP_RK1_OBS>(p, cfg, a, s) : dispatch_pass<R, OP_RK1>(p, cfg, a, s); break;
    case 2: e = dispatch_pass<R, OP_RK2>(p, cfg, a, s); break;
    case 3: e = dispatch_pass<R, OP_RK3>(p, cfg, a, s); break;
    default: e = dispatch_pass<R, OP_RK4>(p, cfg, a, s); break;
  }
  timing_after(fam, s);
  return e;
}

template <typename R>
hipError_t run_rk_stage2_fold(const Plan& p, const LaunchConfig& cfg, const void* Y, const void* y0, const void* field,
                              void* y3, void* A, int64_t step, hipStream_t s) {
  using C = typename CT<R>::T;
  PassArgs<R> a = pass_args<R>();
  a.Y = (const C*)Y;
  a.a = (const C*)y0;
  a.field = (const R*)field;
  a.out = (C*)y3;
  a.out2 = (C*)A;
  a.c_stage = 0.5;
  a.step = step;
  timing_before(FAM_RK2, s);
  hipError_t e = dispatch_pass<R, OP_RK2F>(p, cfg, a, s);
  timing_after(FAM_RK2, s);
  return e;
}

template <typename R>
hipError_t run_rk_stage4_fold(const Plan& p, const LaunchConfig& cfg, const void* Y, const void* A, const void* field,
                              void* out, int64_t step, hipStream_t s) {
  using C = typename CT<R>::T;
  PassArgs<R> a = pass_args<R>();
  a.Y = (const C*)Y;
  a.a = (const C*)A;
  a.field = (const R*)field;
  a.out = (C*)out;
  a.c_stage = 1.0;
  a.step = step;
  timing_before(FAM_RK4, s);
  hipError_t e = dispatch_pass<R, OP_RK4F>(p, cfg, a, s);
  timing_after(FAM_RK4, s);
  return e;
}

template <typename R>
hipError_t run_rk_generic(const Plan& p, const LaunchConfig& cfg, const void* Y, double ccur, int nh,
                          const void* const* hist, const double* hc, double cdt, double c_stage, const void* field,
                          void* out, int64_t step, hipStream_t s) {
  using C = typename CT<R>::T;
  if (nh < 0 || nh > RKG_MAX_HIST) return hipErrorInvalidValue;
  PassArgs<R> a = pass_args<R>();
  a.Y = (const C*)Y;
  a.field = (const R*)field;
  a.out = (C*)out;
  a.c_stage = c_stage;
  a.step = step;
  a.nh = nh;
  for (int j = 0; j < nh; ++j) {
    a.h[j] = (const C*)hist[j];
    a.hc[j] = hc[j];
  }
  a.ccur = ccur;
  a.cdt = cdt;
  timing_before(FAM_RKG, s);
  hipError_t e = dispatch_pass<R, OP_RKG>(p, cfg, a, s);
  timing_after(FAM_RKG, s);
  return e;
}

template <typename R>
hipError_t run_observe(const Plan& p, const LaunchConfig& cfg, const void* psi, const void* field,
                       double t_offset_steps, bool use_scale, int64_t step, hipStream_t s, bool real) {
  using C = typename CT<R>::T;
  PassArgs<R> a = pass_args<R>();
  a.Y = (const C*)psi;
  a.field = (const R*)field;
  a.c_stage = t_offset_steps;
  a.step = step;
  a.use_scale = use_scale ? 1 : 0;
  timing_before(FAM_OBSERVE, s);
  hipError_t e = real ? dispatch_pass<R, OP_OBS, true>(p, cfg, a, s) : dispatch_pass<R, OP_OBS>(p, cfg, a, s);
  timing_after(FAM_OBSERVE, s);
  return e;
}

template <typename R>
hipError_t run_adj_stage(const Plan& p, const LaunchConfig& cfg, int stage, const void* X, const void* Y,
                         const void* field, const void* lam, void* lacc, void* uout, int64_t step, hipStream_t s) {
  using C = typename CT<R>::T;
  PassArgs<R> a = pass_args<R>();
  a.Y = (const C*)X;
  a.a = (const C*)Y;
  a.b = (const C*)lam;
  a.field = (const R*)field;
  a.out = (C*)uout;
  a.out2 = (C*)lacc;
  static const double cst[4] = {0.0, 0.5, 0.5, 1.0};
  if (stage < 1 || stage > 4) return hipErrorInvalidValue;
  a.c_stage = cst[stage - 1];
  a.step = step;
  const int fam = FAM_ADJ1 + stage - 1;
  timing_before(fam, s);
  hipError_t e;
  switch (stage) {
    case 4: e = dispatch_pass<R, OP_ADJ4>(p, cfg, a, s); break;
    case 3: e = dispatch_pass<R, OP_ADJ3>(p, cfg, a, s); break;
    case 2: e = dispatch_pass<R, OP_ADJ2>(p, cfg, a, s); break;
    default: e = dispatch_pass<R, OP_ADJ1>(p, cfg, a, s); break;
  }
  timing_after(fam, s);
  return e;
}

// ---------------------------------------------------------------------------
// pointwise passes (one workgroup of 256 lanes per chunk)
// ---------------------------------------------------------------------------
// PT_PHI / PT_PHI_REAL: the first diagonal half-step of an imaginary-time
// step on its own, phi = s psi P (1 - g |s psi|^2 dt/2) (P read from `field`)
enum PointOp { PT_PROP = 0, PT_SCALE, PT_OVERLAP, PT_SEED, PT_RANGE, PT_SCALE_REAL, PT_PHI, PT_PHI_REAL };

template <typename R> struct PointArgs {
  using C = typename CT<R>::T;
  const C* a;
  const C* b;
  const R* field;
  const R* rin;
  C* out;
  R* rout;
};

template <typename R, int OP>
__global__ __launch_bounds__(256) void k_point(const Plan pl, const PointArgs<R> a) {
  using C = typename CT<R>::T;
  constexpr int NR = OP == PT_RANGE ? 3 : (OP == PT_OVERLAP ? 2 : 1);
  __shared__ double red[4][NR];
  const int cidx = (int)blockIdx.x;
  const Chunk ch = pl.chunks[cidx];
  const InstParams& ip = pl.inst[ch.inst];
  const int kind = ip.pot_kind;
  const R omega2 = (R)pot_const(ip);
  const double t = ip.t0 + (double)(*pl.step) * ip.dt;
  const R delta = (R)pot_param(ip, t);
  const R* const field2 = reinterpret_cast<const R*>(ip.field2);
  double acc[NR];
  if (OP == PT_RANGE) {
    acc[0] = 1e300;
    acc[1] = -1e300;
    acc[2] = 0.0;
  } else {
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0.0;
  }
  R sc = R(1);
  double cre = 0.0, cim = 0.0;
  if (OP == PT_SCALE || OP == PT_SCALE_REAL || OP == PT_PHI || OP == PT_PHI_REAL) sc = (R)pl.out[ch.inst].scale;
  const R hg = (R)ip.g * (R)ip.dt * R(0.5);
  if (OP == PT_SEED) {
    cre = pl.out[ch.inst].ov_re;
    cim = pl.out[ch.inst].ov_im;
  }
  for (int l = threadIdx.x; l < ch.count; l += 256) {
    const int64_t s = (int64_t)ch.site_begin + l;
    if constexpr (OP == PT_PROP) {
      const R V = potential<R>(kind, a.field[s], kind == GPE_POT_LERP ? field2[s] : R(0), delta, omega2);
      a.rout[s] = exp(-V * (R)ip.dt * R(0.5));
    } else if constexpr (OP == PT_SCALE) {
      const C v = a.out[s];
      a.out[s] = cmk<R>(v.x * sc, v.y * sc);
    } else if constexpr (OP == PT_SCALE_REAL) {
      a.rout[s] = a.rout[s] * sc;
    } else if constexpr (OP == PT_PHI) {
      const C v = a.a[s];
      const R vr = v.x * sc, vi = v.y * sc;
      const R f = a.field[s] * (R(1) - hg * (vr * vr + vi * vi));
      a.out[s] = cmk<R>(vr * f, vi * f);
    } else if constexpr (OP == PT_PHI_REAL) {
      const R vr = a.rin[s] * sc;
      a.rout[s] = vr * (a.field[s] * (R(1) - hg * vr * vr));
    } else if constexpr (OP == PT_OVERLAP) {
      const C x = a.a[s], y = a.b[s];
      acc[0] += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
      acc[1] += (double)x.x * (double)y.y - (double)x.y * (double)y.x;
    } else if constexpr (OP == PT_SEED) {
      // lambda_N = -2 dV c psi_target
      const C x = a.a[s];
      const double f = -2.0 * ip.dV;
      a.out[s] = cmk<R>((R)(f * (cre * x.x - cim * x.y)), (R)(f * (cre * x.y + cim * x.x)));
    } else if constexpr (OP == PT_RANGE) {
      const double u = (double)a.field[s];
      acc[0] = u < acc[0] ? u : acc[0];
      acc[1] = u > acc[1] ? u : acc[1];
      // largest density of the state (a: complex, rin: real); NaN propagates
      double d = 0.0;
      if (a.a) {
        const C v = a.a[s];
        d = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
      } else if (a.rin) {
        d = (double)a.rin[s] * (double)a.rin[s];
      }
      acc[2] = (d > acc[2] || d != d) ? d : acc[2];
    }
  }
  if constexpr (OP == PT_OVERLAP) {
    block_sum<256, NR>(acc, red);
    if (threadIdx.x == 0)
      for (int r = 0; r < NR; ++r) pl.partials[(size_t)r * pl.pstride + cidx] = acc[r];
  } else if constexpr (OP == PT_RANGE) {
    for (int off = 32; off > 0; off >>= 1) {
      const double lo = __shfl_xor(acc[0], off, 64), hi = __shfl_xor(acc[1], off, 64);
      const double dm = __shfl_xor(acc[2], off, 64);
      acc[0] = lo < acc[0] ? lo : acc[0];
      acc[1] = hi > acc[1] ? hi : acc[1];
      acc[2] = (dm > acc[2] || dm != dm) ? dm : acc[2];
    }
    if ((threadIdx.x & 63) == 0) {
      red[threadIdx.x >> 6][0] = acc[0];
      red[threadIdx.x >> 6][1] = acc[1];
      red[threadIdx.x >> 6][2] = acc[2];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double lo = red[0][0], hi = red[0][1], dm = red[0][2];
      for (int w = 1; w < 4; ++w) {
        lo = red[w][0] < lo ? red[w][0] : lo;
        hi = red[w][1] > hi ? red[w][1] : hi;
        dm = (red[w][2] > dm || red[w][2] != red[w][2]) ? red[w][2] : dm;
      }
      pl.partials[cidx] = lo;
      pl.partials[(size_t)pl.pstride + cidx] = hi;
      pl.partials[(size_t)2 * pl.pstride + cidx] = dm;
    }
  }
}

template <typename R, int OP>
static hipError_t launch_point(const Plan& p, const PointArgs<R>& a, hipStream_t s) {
  if (p.n_chunks <= 0) return hipSuccess;
  timing_before(FAM_POINTWISE, s);
  hipLaunchKernelGGL((k_point<R, OP>), dim3(p.n_chunks), dim3(256), 0, s, p, a);
  hipError_t e = hipGetLastError();
  timing_after(FAM_POINTWISE, s);
  return e;
}

template <typename R> static PointArgs<R> point_args() {
  PointArgs<R> a;
  a.a = a.b = nullptr;
  a.field = nullptr;
  a.rin = nullptr;
  a.out = nullptr;
  a.rout = nullptr;
  return a;
}

template <typename R>
hipError_t run_make_prop(const Plan& p, const LaunchConfig&, const void* field, void* prop, hipStream_t s) {
  PointArgs<R> a = point_args<R>();
  a.field = (const R*)field;
  a.rout = (R*)prop;
  return launch_point<R, PT_PROP>(p, a, s);
}

template <typename R>
hipError_t run_apply_scale(const Plan& p, const LaunchConfig&, void* psi, bool real, hipStream_t s) {
  PointArgs<R> a = point_args<R>();
  if (real) {
    a.rout = (R*)psi;
    return launch_point<R, PT_SCALE_REAL>(p, a, s);
  }
  a.out = (typename CT<R>::T*)psi;
  return launch_point<R, PT_SCALE>(p, a, s);
}

template <typename R>
hipError_t run_itp_phi(const Plan& p, const LaunchConfig&, const void* psi, const void* prop, void* phi, bool real,
                       hipStream_t s) {
  PointArgs<R> a = point_args<R>();
  a.field = (const R*)prop;
  if (real) {
    a.rin = (const R*)psi;
    a.rout = (R*)phi;
    return launch_point<R, PT_PHI_REAL>(p, a, s);
  }
  a.a = (const typename CT<R>::T*)psi;
  a.out = (typename CT<R>::T*)phi;
  return launch_point<R, PT_PHI>(p, a, s);
}

template <typename R>
hipError_t run_overlap(const Plan& p, const LaunchConfig&, const void* x, const void* y, hipStream_t s) {
  PointArgs<R> a = point_args<R>();
  a.a = (const typename CT<R>::T*)x;
  a.b = (const typename CT<R>::T*)y;
  return launch_point<R, PT_OVERLAP>(p, a, s);
}

template <typename R>
hipError_t run_seed_lambda(const Plan& p, const LaunchConfig&, const void* target, void* lam, hipStream_t s) {
  PointArgs<R> a = point_args<R>();
  a.a = (const typename CT<R>::T*)target;
  a.out = (typename CT<R>::T*)lam;
  return launch_point<R, PT_SEED>(p, a, s);
}

template <typename R>
hipError_t run_field_range(const Plan& p, const LaunchConfig&, const void* field, const void* psi, hipStream_t s,
                           bool real_psi) {
  PointArgs<R> a = point_args<R>();
  a.field = (const R*)field;
  if (real_psi) a.rin = (const R*)psi;
  else a.a = (const typename CT<R>::T*)psi;
  return launch_point<R, PT_RANGE>(p, a, s);
}

// ---------------------------------------------------------------------------
// finalize: one workgroup per instance sums its chunks' partials in order
// ---------------------------------------------------------------------------
constexpr int FIN_BLOCK = 1024;

__global__ __launch_bounds__(FIN_BLOCK) void k_finalize(const Plan pl, int kind, gpe_obs* obs_dev) {
  __shared__ double red[FIN_BLOCK / 64][NPART];
  const int inst = (int)blockIdx.x;
  const InstParams& ip = pl.inst[inst];
  if (kind == FIN_LOSS) {
    if (threadIdx.x == 0) {
      InstOut& o = pl.out[inst];
      o.loss = 1.0 - (o.ov_re * o.ov_re + o.ov_im * o.ov_im);
    }
    return;
  }
  const int c0 = ip.chunk_begin, c1 = ip.chunk_begin + ip.chunk_count;
  const size_t ps = (size_t)pl.pstride;
  const bool range = (kind == FIN_RANGE);
  const int nr = (kind == FIN_OBS) ? 4 : ((kind == FIN_NORM_SCALE) ? 1 : (range ? 3 : 2));
  double acc[NPART];
  acc[0] = range ? 1e300 : 0.0;
  acc[1] = range ? -1e300 : 0.0;
  acc[2] = acc[3] = 0.0;
  // component-major partials: each pass of the loop is a coalesced read; 8
  // independent loads are issued before they are added in a fixed order
  // (with 32 the 1024-lane block runs out of registers and spills)
  constexpr int U = 8;
  for (int base = c0; base < c1; base += FIN_BLOCK * U) {
    for (int r = 0; r < nr; ++r) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = base + (int)threadIdx.x + u * FIN_BLOCK;
        v[u] = (c < c1) ? pl.partials[r * ps + c] : (range ? (r == 0 ? 1e300 : (r == 1 ? -1e300 : 0.0)) : 0.0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (range)
          acc[r] = (r == 0) ? (v[u] < acc[r] ? v[u] : acc[r])
                            : ((v[u] > acc[r] || (r == 2 && v[u] != v[u])) ? v[u] : acc[r]);
        else
          acc[r] += v[u];
      }
    }
  }
  if (range) {
    for (int off = 32; off > 0; off >>= 1) {
      const double lo = __shfl_xor(acc[0], off, 64), hi = __shfl_xor(acc[1], off, 64);
      const double dm = __shfl_xor(acc[2], off, 64);
      acc[0] = lo < acc[0] ? lo : acc[0];
      acc[1] = hi > acc[1] ? hi : acc[1];
      acc[2] = (dm > acc[2] || dm != dm) ? dm : acc[2];
    }
    if ((threadIdx.x & 63) == 0) {
      red[threadIdx.x >> 6][0] = acc[0];
      red[threadIdx.x >> 6][1] = acc[1];
      red[threadIdx.x >> 6][2] = acc[2];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double lo = red[0][0], hi = red[0][1], dm = red[0][2];
      for (int w = 1; w < FIN_BLOCK / 64; ++w) {
        lo = red[w][0] < lo ? red[w][0] : lo;
        hi = red[w][1] > hi ? red[w][1] : hi;
        dm = (red[w][2] > dm || red[w][2] != red[w][2]) ? red[w][2] : dm;
      }
      pl.out[inst].fmin = lo;
      pl.out[inst].fmax = hi;
      pl.out[inst].dmax = dm;
    }
    return;
  }
  block_sum<FIN_BLOCK, NPART>(acc, red);
  if (threadIdx.x != 0) return;
  InstOut& o = pl.out[inst];
  const double dV = ip.dV;
  if (kind == FIN_NORM_SCALE) {
    const double n = dV * acc[0];
    o.norm = n;
    o.scale = sqrt(ip.norm_target / n);
  } else if (kind == FIN_OBS) {
    const double N = dV * acc[0];
    const double E = dV * (acc[1] + acc[2] + 0.5 * ip.g * acc[3]) / N;
    const double mu = dV * (acc[1] + acc[2] + ip.g * acc[3]) / N;
    o.norm = N;
    o.energy = E;
    o.mu = mu;
    if (obs_dev) {
      obs_dev[inst].norm = N;
      obs_dev[inst].energy = E;
      obs_dev[inst].mu = mu;
    }
  } else if (kind == FIN_OVERLAP) {
    o.ov_re = dV * acc[0];
    o.ov_im = dV * acc[1];
  }
}

hipError_t run_finalize(const Plan& p, int kind, gpe_obs* obs_dev, hipStream_t s) {
  timing_before(FAM_FINALIZE, s);
  hipLaunchKernelGGL(k_finalize, dim3(p.n_inst), dim3(FIN_BLOCK), 0, s, p, kind, obs_dev);
  hipError_t e = hipGetLastError();
  timing_after(FAM_FINALIZE, s);
  return e;
}

__global__ __launch_bounds__(64) void k_knot_finalize(const Plan pl, double* grads) {
  const int inst = (int)blockIdx.x;
  const InstParams& ip = pl.inst[inst];
  const int k = (int)threadIdx.x;
  if (k >= GPE_MAX_KNOTS) return;
  double s = 0.0;
  for (int c = ip.chunk_begin; c < ip.chunk_begin + ip.chunk_count; ++c) s += pl.knot_acc[(size_t)c * GPE_MAX_KNOTS + k];
  grads[(size_t)inst * GPE_MAX_KNOTS + k] = s;
}

hipError_t run_knot_finalize(const Plan& p, double* grads_dev, hipStream_t s) {
  timing_before(FAM_FINALIZE, s);
  hipLaunchKernelGGL(k_knot_finalize, dim3(p.n_inst), dim3(64), 0, s, p, grads_dev);
  hipError_t e = hipGetLastError();
  timing_after(FAM_FINALIZE, s);
  return e;
}

__global__ void k_zero_doubles(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

hipError_t run_zero_doubles(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero_doubles, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

__global__ void k_set_scale_one(const Plan pl) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < pl.n_inst) pl.out[i].scale = 1.0;
}

hipError_t run_set_scale_one(const Plan& p, hipStream_t s) {
  hipLaunchKernelGGL(k_set_scale_one, dim3((p.n_inst + 63) / 64), dim3(64), 0, s, p);
  return hipGetLastError();
}

__global__ void k_set_step(int64_t* step, int64_t value) {
  if (threadIdx.x == 0) *step = value;
}
__global__ void k_tick(int64_t* step, int64_t delta) {
  if (threadIdx.x == 0) *step += delta;
}

hipError_t run_set_step(int64_t* step, int64_t value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, step, value);
  return hipGetLastError();
}

hipError_t run_tick(int64_t* step, int64_t delta, hipStream_t s) {
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, step, delta);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// box <-> compact
// ---------------------------------------------------------------------------
template <typename E>
__global__ void k_pack(const int64_t* run_base, const int32_t* run_start, int64_t nruns, int64_t n,
                       const E* src, E* dst, int to_box) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = nruns - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (run_start[mid] <= s) lo = mid; else hi = mid - 1;
    }
    const int64_t box = run_base[lo] + (s - run_start[lo]);
    if (to_box) dst[box] = src[s];
    else dst[s] = src[box];
  }
}

template <typename R>
hipError_t run_pack(const int64_t* run_base, const int32_t* run_start, int64_t nruns, int64_t n_active,
                    const void* src, void* dst, bool to_box, hipStream_t s, bool real) {
  using C = typename CT<R>::T;
  int64_t blocks = (n_active + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  timing_before(FAM_POINTWISE, s);
  if (real)
    hipLaunchKernelGGL((k_pack<R>), dim3((unsigned)blocks), dim3(256), 0, s, run_base, run_start, nruns, n_active,
                       (const R*)src, (R*)dst, to_box ? 1 : 0);
  else
    hipLaunchKernelGGL((k_pack<C>), dim3((unsigned)blocks), dim3(256), 0, s, run_base, run_start, nruns, n_active,
                       (const C*)src, (C*)dst, to_box ? 1 : 0);
  hipError_t e = hipGetLastError();
  timing_after(FAM_POINTWISE, s);
  return e;
}

// Post-selection (Sec. II.A, repeated per ramp stage in Sec. V): the active
// set is min(Va, Vb) < cutoff over the whole box (Vb may be null), found
// directly as z-runs.  One wave per (i, j) column reads the column 64 points
// at a time; the ballot of the selection is compared with itself shifted by
// one point, and every change (a run's first point or the first point after
// it) is taken in order.  The count pass writes the number of runs per
// column; the emit pass writes the runs from the column's offset.
template <typename R>
__global__ __launch_bounds__(256) void k_column_runs(const R* va, const R* vb, int64_t n1, int64_t n01, int64_t n2,
                                                     R cutoff, int32_t* counts, const int64_t* offsets,
                                                     int64_t* runs) {
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < n01; c += nwaves) {
    const int64_t base = c * n2;
    unsigned long long prev = 0;     // selection at k = kk - 1
    bool in_run = false;
    int64_t k0 = 0, nr = 0, pos = offsets ? offsets[c] : 0;
    for (int64_t kk = 0; kk < n2; kk += 64) {
      const int64_t k = kk + lane;
      bool on = false;
      if (k < n2) {
        R v = va[base + k];
        if (vb) {
          const R w = vb[base + k];
          v = w < v ? w : v;
        }
        on = v < cutoff;
      }
      const unsigned long long m = __ballot(on);
      unsigned long long t = m ^ ((m << 1) | prev);
      prev = m >> 63;
      if (!offsets) {
        nr += __popcll(t & m);
        continue;
      }
      while (t) {
        const int64_t kt = kk + (__ffsll((long long)t) - 1);
        t &= t - 1;
        if (!in_run) {
          k0 = kt;
        } else if (lane == 0) {
          int64_t* r = runs + 4 * pos;
          r[0] = c / n1;
          r[1] = c % n1;
          r[2] = k0;
          r[3] = kt;
        }
        if (in_run) ++pos;
        in_run = !in_run;
      }
    }
    if (!offsets) {
      if (lane == 0) counts[c] = (int32_t)nr;
    } else if (in_run && lane == 0) {
      int64_t* r = runs + 4 * pos;
      r[0] = c / n1;
      r[1] = c % n1;
      r[2] = k0;
      r[3] = n2;
    }
  }
}

template <typename R>
hipError_t run_column_runs(const void* va, const void* vb, int64_t n0, int64_t n1, int64_t n2, double cutoff,
                           int32_t* counts, const int64_t* offsets, int64_t* runs, hipStream_t s) {
  const int64_t n01 = n0 * n1;
  if (n01 <= 0 || n2 <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n01 + 3) / 4, 65536);
  hipLaunchKernelGGL((k_column_runs<R>), dim3((unsigned)blocks), dim3(256), 0, s, (const R*)va, (const R*)vb, n1,
                     n01, n2, (R)cutoff, counts, offsets, runs);
  return hipGetLastError();
}

// Carry psi between two compact layouts of one box: the destination array is
// cut into intervals (iv_dst[q] = first destination site, sorted, iv_dst[0]
// = 0), each copied from consecutive source sites starting at iv_src[q] or
// zero-filled when iv_src[q] < 0.  One wave per interval (grid-stride over
// the intervals) copies it with consecutive lanes on consecutive sites.
template <typename R>
__global__ __launch_bounds__(256) void k_remap(const int64_t* iv_dst, const int64_t* iv_src, int64_t n_iv,
                                               int64_t n_dst, const typename CT<R>::T* src,
                                               typename CT<R>::T* dst) {
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t q = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); q < n_iv; q += nwaves) {
    const int64_t d0 = iv_dst[q], d1 = q + 1 < n_iv ? iv_dst[q + 1] : n_dst, o = iv_src[q];
    for (int64_t i = d0 + lane; i < d1; i += 64) dst[i] = o >= 0 ? src[o + (i - d0)] : cmk<R>(R(0), R(0));
  }
}

// one 16-byte load and one 16-byte store per lane, nothing else
__global__ __launch_bounds__(256) void k_stream_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                                                     size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t run_stream_copy(const void* src, void* dst, size_t n16, hipStream_t s) {
  if (n16 == 0) return hipSuccess;
  timing_before(FAM_COPY, s);
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, s, (const double2*)src,
                     (double2*)dst, n16);
  hipError_t e = hipGetLastError();
  timing_after(FAM_COPY, s);
  return e;
}

template <typename R>
hipError_t run_remap(const int64_t* iv_dst, const int64_t* iv_src, int64_t n_iv, int64_t n_dst, const void* src,
                     void* dst, hipStream_t s) {
  using C = typename CT<R>::T;
  if (n_dst <= 0 || n_iv <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n_iv + 3) / 4, 65536);
  timing_before(FAM_POINTWISE, s);
  hipLaunchKernelGGL((k_remap<R>), dim3((unsigned)blocks), dim3(256), 0, s, iv_dst, iv_src, n_iv, n_dst,
                     (const C*)src, (C*)dst);
  hipError_t e = hipGetLastError();
  timing_after(FAM_POINTWISE, s);
  return e;
}

template <typename R>
__global__ void k_fill_zero(typename CT<R>::T* d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = cmk<R>(R(0), R(0));
}

template <typename R>
hipError_t run_fill_zero(void* dst, int64_t n, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL((k_fill_zero<R>), dim3((unsigned)blocks), dim3(256), 0, s, (typename CT<R>::T*)dst, n);
  return hipGetLastError();
}

// explicit instantiations
#define GPE_INST(R)                                                                                            \
  template hipError_t run_itp_pass1<R>(const Plan&, const LaunchConfig&, const void*, const void*, void*,    \
                                       bool, hipStream_t, bool, bool);                                       \
  template hipError_t run_itp_phi<R>(const Plan&, const LaunchConfig&, const void*, const void*, void*, bool,  \
                                     hipStream_t);                                                           \
  template hipError_t run_itp_pass2<R>(const Plan&, const LaunchConfig&, const void*, const void*, void*,    \
                                       bool, hipStream_t);                                                   \
  template hipError_t run_rk_stage<R>(const Plan&, const LaunchConfig&, int, bool, const void*, const void*, \
                                      const void*, const void*, const void*, void*, int64_t, hipStream_t);   \
  template hipError_t run_rk_stage2_fold<R>(const Plan&, const LaunchConfig&, const void*, const void*,       \
                                            const void*, void*, void*, int64_t, hipStream_t);                \
  template hipError_t run_rk_stage4_fold<R>(const Plan&, const LaunchConfig&, const void*, const void*,       \
                                            const void*, void*, int64_t, hipStream_t);                       \
  template hipError_t run_rk_generic<R>(const Plan&, const LaunchConfig&, const void*, double, int,            \
                                        const void* const*, const double*, double, double, const void*, void*, \
                                        int64_t, hipStream_t);                                                \
  template hipError_t run_observe<R>(const Plan&, const LaunchConfig&, const void*, const void*, double, bool, \
                                     int64_t, hipStream_t, bool);                                            \
  template hipError_t run_adj_stage<R>(const Plan&, const LaunchConfig&, int, const void*, const void*,      \
                                       const void*, const void*, void*, void*, int64_t, hipStream_t);        \
  template hipError_t run_make_prop<R>(const Plan&, const LaunchConfig&, const void*, void*, hipStream_t);   \
  template hipError_t run_apply_scale<R>(const Plan&, const LaunchConfig&, void*, bool, hipStream_t);        \
  template hipError_t run_overlap<R>(const Plan&, const LaunchConfig&, const void*, const void*, hipStream_t); \
  template hipError_t run_seed_lambda<R>(const Plan&, const LaunchConfig&, const void*, void*, hipStream_t); \
  template hipError_t run_field_range<R>(const Plan&, const LaunchConfig&, const void*, const void*,          \
                                         hipStream_t, bool);                                                 \
  template hipError_t run_pack<R>(const int64_t*, const int32_t*, int64_t, int64_t, const void*, void*, bool, \
                                  hipStream_t, bool);                                                        \
  template hipError_t run_fill_zero<R>(void*, int64_t, hipStream_t);                                         \
  template hipError_t run_column_runs<R>(const void*, const void*, int64_t, int64_t, int64_t, double, int32_t*, \
                                         const int64_t*, int64_t*, hipStream_t);                             \
  template hipError_t run_remap<R>(const int64_t*, const int64_t*, int64_t, int64_t, const void*, void*,      \
                                   hipStream_t);

GPE_INST(double)
GPE_INST(float)

}  // namespace gpe
