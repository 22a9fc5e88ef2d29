/*
 * gpe.h - C ABI of the MI355X (gfx950) solver for the Gross-Pitaevskii
 * equation on a selectively sampled, semi-structured grid.
 *
 * Method: Beregi, Gerent, Lundblad, "Efficient simulation of Bose-Einstein
 * condensates in nontrivial topologies" (arXiv:2603.05447).
 *
 * Problem (Sec. II, eqs. (1)-(3)), hbar = m = 1:
 *   i d(psi)/dt = -1/2 Lap psi + V(x,t) psi + g |psi|^2 psi,   dV sum |psi|^2 = N.
 * The grid is a Cartesian box of n[0] x n[1] x n[2] points at spacing h;
 * only the sites of an active set A (the region of interest of Sec. II.A,
 * e.g. the Thomas-Fermi region {V < cutoff}) are stored.  Rows/columns of
 * the 7-point Laplacian (App. B, eq. (B1)) outside A are removed, i.e. psi
 * is zero (Dirichlet) outside A and outside the box.
 *
 * Layout conventions used by every call:
 *   - site (i,j,k) sits at x0 + (i,j,k).*h; box linear index (i*n1 + j)*n2 + k
 *     (z fastest);
 *   - "compact" arrays hold one entry per active site, in increasing box
 *     linear index order; n_active < 2^31;
 *   - complex arrays are interleaved (re, im): GPE_C128 = 2 x double per
 *     site, GPE_C64 = 2 x float per site; real per-site arrays (potential
 *     fields) use double for GPE_C128 and float for GPE_C64;
 *   - device pointers are caller-owned and must be 16-byte aligned; the
 *     library never frees them;
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls
 *     are stream-ordered and asynchronous, except that a call writing to a
 *     *_host output synchronises `stream` before returning.  A grid or batch
 *     keeps per-handle device state (instance table, reduction partials,
 *     results, step counter), so the work of a call on a handle starts after
 *     the work of the previous call on the same handle, whichever stream that
 *     one used (the library makes the new stream wait for the old one's last
 *     event; not applied while `stream` is being captured into a graph).
 *     Caller-owned buffers (psi, fields, work) are the caller's to order.
 *
 * Errors: every call returns a gpe_status.  Arguments are validated before
 * anything is launched, so a call that fails validation has no effect.  A
 * failure is described by gpe_last_error() (thread-local, valid until the
 * next gpe_* call on the same thread).  No call aborts or throws.
 * Handles must not be used from several threads at once.
 */
#ifndef GPE_H
#define GPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GPE_ABI_VERSION 4
#define GPE_MAX_KNOTS 32

typedef enum {
  GPE_OK = 0,
  GPE_ERR_ARG = 1,        /* invalid argument (null pointer, bad size, bad geometry, ...) */
  GPE_ERR_ALLOC = 2,      /* host or device allocation failed */
  GPE_ERR_DEVICE = 3,     /* a HIP call failed (including a device fault surfacing at a sync) */
  GPE_ERR_STATE = 4,      /* handle not usable for this call (e.g. a host-only grid) */
  GPE_ERR_UNSTABLE = 5,   /* dt above the explicit-scheme stability bound (checked unless skipped) */
  GPE_ERR_NONFINITE = 6   /* a norm observed during the run was NaN/Inf */
} gpe_status;

typedef enum { GPE_C128 = 0, GPE_C64 = 1 } gpe_dtype;

typedef enum {
  GPE_MODE_ITP = 0,       /* gpe_imag_time */
  GPE_MODE_RT = 1,        /* gpe_real_time with GPE_RK4 */
  GPE_MODE_ADJ = 2,       /* gpe_fidelity_grad */
  GPE_MODE_RT_RKHE3 = 3,  /* gpe_real_time with GPE_RKHE3 */
  GPE_MODE_RT_RKCK = 4,   /* gpe_real_time with GPE_RKCK */
  GPE_MODE_ITP_REAL = 5   /* gpe_imag_time_real */
} gpe_mode;

/* Explicit integrators for real time (Sec. II.A; App. A gives each one's
 * memory-optimised form): the classic fourth-order method, Heun's
 * third-order method and the fifth-order Cash-Karp weights. */
typedef enum { GPE_RK4 = 0, GPE_RKHE3 = 1, GPE_RKCK = 2 } gpe_integrator;

typedef struct {
  int64_t n[3];   /* points per axis, each >= 1 */
  double h[3];    /* spacing per axis, each > 0 */
  double x0[3];   /* coordinates of site (0,0,0) */
} gpe_geometry;

typedef struct gpe_grid_s* gpe_grid;
typedef struct gpe_batch_s* gpe_batch;

/* Potential (Sec. V, eq. (10)).
 *   STATIC : V(x) = field[x].
 *   RF_RAMP: V(x,t) = sqrt((field[x] - Delta(t))^2 + omega^2), the RF-dressed
 *            potential with bare trap U = field; Delta(t) is the
 *            piecewise-linear interpolant of (knot_t[k], knot_delta[k]),
 *            constant before the first and after the last knot.
 *   SHELL_RAMP: V(x,t) = omega/2 (field[x] - R0(t))^2, a harmonic shell of
 *            stiffness lambda = omega around the distances r = field (the
 *            shell of the C1 workload) whose radius R0(t) is ramped like
 *            Delta(t): the piecewise-linear interpolant of (knot_t[k],
 *            knot_delta[k] = R0_k).  Used by every call that takes RF_RAMP.
 *   LERP   : one stage of a staged ramp (Sec. V: precomputed potentials,
 *            linear interpolation in time between consecutive ones):
 *            V(x,t) = (1 - l) field[x] + l field2[x], l = clamp((t - knot_t[0]) /
 *            (knot_t[1] - knot_t[0]), 0, 1); n_knots = 2, knot_delta unused.
 *            Real time and imaginary time only (not the fidelity gradient
 *            or batches).
 * `field` (and `field2`) are device pointers to n_active reals (double for
 * GPE_C128, float for GPE_C64).  knot_t/knot_delta are host arrays of n_knots
 * (1..GPE_MAX_KNOTS) entries, knot_t strictly increasing; ignored for STATIC.
 * field2 is ignored except for LERP. */
typedef enum { GPE_POT_STATIC = 0, GPE_POT_RF_RAMP = 1, GPE_POT_LERP = 2, GPE_POT_SHELL_RAMP = 3 } gpe_pot_kind;

typedef struct {
  int32_t kind;
  int32_t n_knots;
  const void* field;
  double omega;
  const double* knot_t;
  const double* knot_delta;
  const void* field2;
} gpe_potential;

typedef struct {
  double g;               /* interaction constant of eqs. (1)-(2) */
  double dt;              /* time step, > 0 */
  double norm_target;     /* N of eq. (3) for imaginary time; <= 0 means 1 */
  int64_t obs_every;      /* > 0: record an observation every obs_every steps */
  int32_t skip_stability_check; /* 0 (default): check dt before any step is launched and fail
                                   with GPE_ERR_UNSTABLE above the bound; nonzero: skip the check */
  int32_t integrator;     /* gpe_integrator for real time (0 = GPE_RK4); other calls need 0 */
} gpe_params;

typedef struct { double norm, energy, mu; } gpe_obs;

const char* gpe_last_error(void);
int gpe_abi_version(void);

/* Build the compact layout of a grid (Sec. II.A: flatten, drop the sites
 * outside the region of interest; the "normal point" structure of the
 * paper's CPU kernel, generalised to runs along z split into segments with
 * constant lateral neighbour offsets).
 *   mask_host: n0*n1*n2 bytes, nonzero = active, box linear order.
 *   device   : HIP device ordinal; -1 builds a host-only grid (tables only,
 *              no device memory; compute calls on it return GPE_ERR_STATE).
 * On success *out owns host and device tables; free with gpe_grid_destroy.
 * Errors: GPE_ERR_ARG for bad geometry, an empty active set or more than
 * 2^31-1 active sites; GPE_ERR_ALLOC/GPE_ERR_DEVICE on allocation/copy failure. */
gpe_status gpe_grid_create(const gpe_geometry* geom, const uint8_t* mask_host, int device, gpe_grid* out);

/* Same, from a host list of z-runs: runs_host holds nruns x {i, j, k0, k1}
 * (int64, k1 exclusive), sorted by (i, j, k0), non-overlapping; runs that
 * touch (k0 == previous k1 in the same column) are merged.  Suitable for
 * boxes whose dense mask would be too large (e.g. 2^32 points). */
gpe_status gpe_grid_create_runs(const gpe_geometry* geom, int64_t nruns, const int64_t* runs_host,
                                int device, gpe_grid* out);

/* Post-selection from potentials on the device (Sec. II.A; repeated at the
 * end of every stage of a staged ramp in Sec. V): the active set is
 * {x : min(va_box[x], vb_box[x]) < cutoff} over the whole box (vb_box may be
 * NULL: va_box alone).  va_box/vb_box are device arrays of n0*n1*n2 reals in
 * box linear order (double for GPE_C128, float for GPE_C64) on `device`
 * (>= 0).  For a stage between potentials V_i and V_{i+1} the paper's cutoff
 * is 5 max(mu_i, mu_{i+1}).  The z-runs of the selection are found on the
 * device (one wave per (i, j) column; no box mask is formed) and only the run
 * table is copied to the host, where the segments are built as in
 * gpe_grid_create_runs; the call runs on the null stream and synchronises
 * (potentials written on a non-blocking stream must be complete before the
 * call).  Errors as gpe_grid_create (an empty selection is GPE_ERR_ARG). */
gpe_status gpe_grid_create_threshold(const gpe_geometry* geom, gpe_dtype dtype, const void* va_box,
                                     const void* vb_box, double cutoff, int device, gpe_grid* out);

/* Carry a wavefunction from one compact layout to another of the same box
 * (Sec. V: psi is remapped from the old grid to the new one at every stage
 * end): every site active in both keeps its value, sites only in `dst` are
 * set to zero, sites only in `src` are dropped.  psi_src holds src's
 * n_active complex values, psi_dst receives dst's; they must not alias.
 * Both grids must be on the same device with the same box dimensions.  The
 * copy is exact (no arithmetic).  The call synchronises `stream`. */
gpe_status gpe_remap(gpe_grid src, gpe_grid dst, gpe_dtype dtype, const void* psi_src, void* psi_dst, void* stream);

gpe_status gpe_grid_info(gpe_grid grid, int64_t* n_active, int64_t* n_runs, int64_t* n_segments);

/* Host copy of the segment table: n_segments x 8 int32 per segment
 * {start, length, flags, off_xm, off_xp, off_ym, off_yp, 0}.  `start` is the
 * compact index of the segment's first site; off_* is the constant compact
 * offset of the (i-1), (i+1), (j-1), (j+1) neighbour of every site of the
 * segment, 0 when that neighbour is outside A; flags bit 0 = the segment
 * begins a z-run (its first site has no k-1 neighbour), bit 1 = it ends a
 * z-run (its last site has no k+1 neighbour). */
gpe_status gpe_grid_segments(gpe_grid grid, int32_t* out_host);

/* Host copy of the run table: n_runs x 5 int64 {i, j, k0, k1, start}. */
gpe_status gpe_grid_runs(gpe_grid grid, int64_t* out_host);

/* Laplacian stencil used by every later call on the grid:
 *   7  (the default) App. B eq. (B1);
 *   19 the higher-order compact stencil of App. B eq. (B2): Lap_7 + (1/12)
 *      sum over axis pairs (a, b) of (h_a^2 + h_b^2) delta_a^2 (x) delta_b^2;
 *   27 the cubic 27-point stencil (Sec. II.B and III use a 3^3 HOC stencil
 *      without printing it): for equal spacings h, (1/(30 h^2)) times
 *      -128 at the centre, 14 at the 6 faces, 3 at the 12 edges and 1 at the
 *      8 corners; like eq. (B2) its leading error is the isotropic
 *      (h^2/12) Lap^2.  Equal spacings are required (GPE_ERR_ARG otherwise).
 * Every stencil is restricted to the active set like Lap_7 (rows and columns
 * outside A removed, i.e. psi = 0 off A).  The 19/27-point tables (16/24
 * lateral taps per segment) are built on first use.  They are available for
 * single grids whose per-site arrays are below 4 GiB; their kernels run 256
 * lanes x 1 site whatever the launch configuration says.  The stability
 * checks use the Gershgorin bound of the selected operator.
 * Errors: GPE_ERR_ARG for another point count. */
gpe_status gpe_grid_set_stencil(gpe_grid grid, int32_t points);
gpe_status gpe_grid_get_stencil(gpe_grid grid, int32_t* points);

/* Host copy of the 19- or 27-point segment table (built on demand, also for
 * host-only grids): *n_segments rows of 4 + T int32 {start, length, flags,
 * off[T], 0}, T = 16 (points = 19) or 24 (points = 27); off[t] is the
 * constant compact offset of lateral tap t (0 = absent), taps as (di, dj, dk)
 *   (-1,0,0) (1,0,0) (0,-1,0) (0,1,0)  (-1,0,-1) (-1,0,1) (1,0,-1) (1,0,1)
 *   (0,-1,-1) (0,-1,1) (0,1,-1) (0,1,1)  (-1,-1,0) (-1,1,0) (1,-1,0) (1,1,0)
 * and for 27 points the corners (-1,-1,-1) (-1,-1,1) (-1,1,-1) (-1,1,1)
 * (1,-1,-1) (1,-1,1) (1,1,-1) (1,1,1).  out_host may be NULL to query the
 * count only. */
gpe_status gpe_grid_stencil_segments(gpe_grid grid, int32_t points, int64_t* n_segments, int32_t* out_host);

/* Frees the grid's host and device tables and its captured graphs, after
 * waiting for the device's outstanding work.  NULL is accepted. */
gpe_status gpe_grid_destroy(gpe_grid grid);

/* Size in bytes of the device work buffer a call needs.
 *   mode GPE_MODE_ITP: gpe_imag_time (two temporaries and P); GPE_MODE_ITP_REAL:
 *   gpe_imag_time_real (the same in reals);
 *   GPE_MODE_RT / _RT_RKHE3 / _RT_RKCK:
 *   gpe_real_time with that integrator (3, 2 and 5 state vectors);
 *   GPE_MODE_ADJ: gpe_fidelity_grad with nsteps and ckpt_every as given. */
gpe_status gpe_work_bytes(gpe_grid grid, gpe_dtype dtype, int32_t mode, int64_t nsteps, int64_t ckpt_every,
                          size_t* bytes);

/* Box <-> compact copies.  box_dev holds n0*n1*n2 complex values of dtype;
 * gpe_unpack writes zeros at inactive box points. */
gpe_status gpe_pack(gpe_grid grid, gpe_dtype dtype, const void* box_dev, void* compact_dev, void* stream);
gpe_status gpe_unpack(gpe_grid grid, gpe_dtype dtype, const void* compact_dev, void* box_dev, void* stream);
/* Box -> compact for a real field (a potential on the full grid, Sec. V's
 * precomputed stage potentials): n0*n1*n2 reals in, n_active reals out
 * (double for GPE_C128, float for GPE_C64). */
gpe_status gpe_pack_real(gpe_grid grid, gpe_dtype dtype, const void* box_dev, void* compact_dev, void* stream);

/* Imaginary-time propagation with renormalisation (Sec. II.A, eqs. (6)-(7)).
 * Each step: psi <- psi exp(-V dt/2)(1 - g|psi|^2 dt/2); two forward-Euler
 * kinetic substeps of dt/2 (chi = phi - dt/2 T phi, twice); the diagonal
 * half-step again; renormalise to dV sum |psi|^2 = norm_target.  The
 * renormalisation factor is reduced in FP64 on the device and applied when
 * the next step loads psi; psi as returned is normalised.  V is taken at
 * time 0 for RF_RAMP.
 *   psi       : device, n_active complex, in/out.
 *   work      : device, >= gpe_work_bytes(.., GPE_MODE_ITP, ..) bytes.
 *   final_host: optional (may be NULL) observation of the returned psi.
 *   history_dev: optional device array of ceil(nsteps/obs_every) gpe_obs,
 *               observation before steps 0, obs_every, ...
 * Stability (unless params->skip_stability_check): dt/2 * lambda_max(T) <= 2
 * for the Euler substeps (lambda_max(T) the Gershgorin bound of the grid's
 * stencil), and g max|psi|^2 dt/2 < 1 at the start state so that the
 * linearised interaction factor stays positive; a violation returns
 * GPE_ERR_UNSTABLE before any step runs.  The check reads psi and the field
 * once on the device and synchronises `stream`. */
gpe_status gpe_imag_time(gpe_grid grid, gpe_dtype dtype, void* psi, const gpe_potential* pot,
                         const gpe_params* params, int64_t nsteps, void* work, size_t work_bytes,
                         void* stream, gpe_obs* final_host, gpe_obs* history_dev);

/* Imaginary time on a real state (Sec. II.A: with a real start, a real
 * potential and real g every step of eqs. (6)-(7) keeps psi real).  Same
 * step, renormalisation, observations and errors as gpe_imag_time, but psi
 * holds n_active reals (double for GPE_C128, float for GPE_C64), halving
 * the state traffic; g is used as given (real).
 *   work: >= gpe_work_bytes(.., GPE_MODE_ITP_REAL, ..) bytes.
 * The result can seed gpe_real_time after conversion to interleaved complex
 * (imaginary parts zero). */
gpe_status gpe_imag_time_real(gpe_grid grid, gpe_dtype dtype, void* psi, const gpe_potential* pot,
                              const gpe_params* params, int64_t nsteps, void* work, size_t work_bytes,
                              void* stream, gpe_obs* final_host, gpe_obs* history_dev);

/* Real-time evolution (Sec. II.A eq. (8)) with params->integrator, in the
 * memory-optimised form of App. A, eqs. (A6)-(A7): each stage reads one
 * stage state through the stencil plus the earlier stored stage states at
 * the same site, and writes the next stage state; the last stage overwrites
 * psi.
 *   GPE_RK4  : stored y2, y3, y4; final b* = (-1/3, 1/3, 2/3, 1/3) plus
 *              dt/6 k4; stage times t + (0, 1/2, 1/2, 1) dt.
 *   GPE_RKHE3: stored y2, y3; stage times t + (0, 1/3, 2/3) dt.
 *   GPE_RKCK : stored y2..y6; stage times t + (0, 1/5, 3/10, 3/5, 1, 7/8) dt.
 * Step n starts at t0 + n dt.  work: gpe_work_bytes of the matching mode.
 * Stability (unless params->skip_stability_check; Gershgorin bound of the
 * frozen-coefficient operator of eq. (8)): dt * lambda <= 2 sqrt(2) (RK4),
 * sqrt(3) (RKHE3) or 1 (RKCK, whose stability function exceeds 1 in modulus
 * on the whole imaginary axis; at 1 the growth per step is below 2.3e-4), with
 * lambda = lambda_max(T) + max|V| + |g| max|psi|^2 (max|V| over the ramp's
 * knots, max|psi|^2 of the start state); a violation returns
 * GPE_ERR_UNSTABLE before any step runs.  The check reads psi and the field
 * once on the device and synchronises `stream`. */
gpe_status gpe_real_time(gpe_grid grid, gpe_dtype dtype, void* psi, const gpe_potential* pot,
                         const gpe_params* params, double t0, int64_t nsteps, void* work, size_t work_bytes,
                         void* stream, gpe_obs* final_host, gpe_obs* history_dev);

/* gpe_real_time for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same steps, kernels and results as gpe_real_time with the grid's launch
 * variant, but the stage states live in a library-owned static device array
 * of gpe_noalloc_scratch_bytes() bytes (64 MiB; each GPU the library runs on
 * holds its own copy until the process ends) instead of a work argument, and
 * no device or host memory is allocated on success (the launch tables of the
 * grid's variant are built when the grid is created or its variant or stencil
 * is chosen).  A grid whose stage states need more (gpe_work_bytes of the
 * integrator's mode: 3 state vectors for RK4, 2 for RKHE3, 5 for RKCK, i.e.
 * about 1.39M active sites in complex128 RK4) gets GPE_ERR_ARG before
 * anything runs.  Nothing in the array needs to start at zero (every stage
 * state is written before it is read).  Every call on a GPU shares that GPU's
 * array, so calls that overlap on one GPU (on different streams, or on
 * different grids) race; calls on one stream are ordered.  Under graph
 * capture pass final_host = NULL and set params->skip_stability_check (both
 * synchronise the stream).  Per-kernel timing (gpe_timing_enable) keeps host
 * bookkeeping and is meant to be off here. */
gpe_status gpe_real_time_noalloc(gpe_grid grid, gpe_dtype dtype, void* psi, const gpe_potential* pot,
                                 const gpe_params* params, double t0, int64_t nsteps, void* stream,
                                 gpe_obs* final_host, gpe_obs* history_dev);
size_t gpe_noalloc_scratch_bytes(void);

/* Particle number (eq. (3)), energy and chemical potential of psi at time t:
 * E = dV[Re psi^H T psi + sum V|psi|^2 + g/2 sum|psi|^4]/N, mu the same with g. */
gpe_status gpe_observe(gpe_grid grid, gpe_dtype dtype, const void* psi, const gpe_potential* pot, double t,
                       double g, void* stream, gpe_obs* out_host);

/* <a|b> = dV sum conj(a) b, written as {re, im} to out_host. */
gpe_status gpe_overlap(gpe_grid grid, gpe_dtype dtype, const void* a, const void* b, void* stream,
                       double* out_host);

/* Fidelity loss L = 1 - |<psi_target|psi(T)>|^2 after nsteps RK4 steps
 * (params->integrator must be GPE_RK4) from
 * psi0 at t0 under an RF_RAMP potential, and dL/dDelta_k for every knot, by
 * the discrete adjoint of the RK4 map (the paper optimises the ramp without
 * gradients, Sec. V; this is the gradient of the same forward scheme).
 * Forward states are checkpointed every ckpt_every steps (0 = ceil(sqrt(nsteps)));
 * the reverse sweep recomputes one segment at a time from its checkpoint,
 * keeping the segment's stage states, so the work buffer holds
 * ceil(nsteps/K) + 4K + 8 state vectors (K = the checkpoint interval).
 * Stability as gpe_real_time, with 3 |g| max|psi0|^2 in lambda (Gershgorin
 * bound of the linearised operator the adjoint stages apply).
 *   psi_final: optional device output of psi(T) (may be NULL).
 *   grad_host: n_knots doubles. */
gpe_status gpe_fidelity_grad(gpe_grid grid, gpe_dtype dtype, const void* psi0, const void* psi_target,
                             const gpe_potential* pot, const gpe_params* params, double t0, int64_t nsteps,
                             int64_t ckpt_every, void* work, size_t work_bytes, void* stream,
                             double* loss_host, double* grad_host, void* psi_final);

/* ---- Staged ramps (Sec. V) ------------------------------------------
 * A ramp given as stage potentials V_0 .. V_S on the whole box (device box
 * arrays, double for GPE_C128, float for GPE_C64) and the chemical potentials
 * mu_0 .. mu_S of their ground states.  Stage i (i = 0 .. S-1) runs on its own
 * grid, the post-selection of Sec. II.A repeated at the stage boundary: the
 * points where min(V_i, V_{i+1}) < cutoff_factor max(mu_i, mu_{i+1}) (the
 * paper's factor is 5), so every potential met during the stage is covered.
 *
 * gpe_staged_ramp_grids builds the S grids (as gpe_grid_create_threshold;
 * fields_box holds n_fields = S + 1 pointers, mus_host S + 1 values,
 * cutoff_factor <= 0 selects 5).  grids_out receives S handles owned by the
 * caller (gpe_grid_destroy each); cutoffs_host (optional) the S cutoffs.  On
 * failure no grid is left allocated and every grids_out entry is NULL. */
gpe_status gpe_staged_ramp_grids(const gpe_geometry* geom, gpe_dtype dtype, int32_t n_fields,
                                 const void* const* fields_box, const double* mus_host, double cutoff_factor,
                                 int device, gpe_grid* grids_out, double* cutoffs_host);

/* Work buffer of gpe_staged_ramp_run: the largest stage's two compact stage
 * potentials plus its real-time work for `integrator`. */
gpe_status gpe_staged_ramp_work_bytes(int32_t n_stages, const gpe_grid* grids, gpe_dtype dtype, int32_t integrator,
                                      size_t* bytes);

/* Runs the S stages in order.  Stage i carries psi over from the previous
 * grid (stage 0: `src` with psi_src) to grids[i] as gpe_remap does (a plain
 * copy when the selection did not change; no renormalisation), packs V_i and
 * V_{i+1} onto grids[i], observes the carried-over state, and takes
 * steps_per_stage real-time steps (params: g, dt, integrator, stability
 * check) from t_i = t0 + i steps_per_stage dt with the LERP potential from V_i
 * at t_i to V_{i+1} at t_{i+1}.  psi_stage[i] (caller-owned, grids[i]'s
 * n_active complex values) receives the state on stage i's grid; the ramp's
 * result is psi_stage[S-1].  records_host: S x 4 doubles per stage {norm
 * after the carry-over, norm, energy and mu at the stage end}.  Synchronises
 * `stream` (every stage reads its observations on the host). */
gpe_status gpe_staged_ramp_run(gpe_grid src, const void* psi_src, int32_t n_stages, const gpe_grid* grids,
                               void* const* psi_stage, gpe_dtype dtype, const void* const* fields_box,
                               const gpe_params* params, double t0, int64_t steps_per_stage, void* work,
                               size_t work_bytes, void* stream, double* records_host);

/* ---- Batched instances ----------------------------------------------
 * A batch concatenates the compact layouts of n grids (instance i occupies
 * compact sites [offsets[i], offsets[i+1])) so one kernel launch advances
 * every instance.  All per-site buffers passed to batch calls (psi, field,
 * psi_target) are concatenated the same way.  Batches use the 7-point
 * stencil whatever stencil the member grids have selected. */
typedef struct {
  double omega;              /* Omega (RF_RAMP) or lambda (SHELL_RAMP) */
  int32_t n_knots;
  int32_t kind;              /* GPE_POT_RF_RAMP (0 is read as RF_RAMP) or GPE_POT_SHELL_RAMP */
  const double* knot_t;      /* host */
  const double* knot_delta;  /* host: Delta_k (RF_RAMP) or R0_k (SHELL_RAMP) */
} gpe_ramp;

gpe_status gpe_batch_create(int32_t n, const gpe_grid* grids, int device, gpe_batch* out);
gpe_status gpe_batch_offsets(gpe_batch batch, int64_t* offsets_host /* n+1 */);
/* As gpe_grid_destroy, for a batch (its grids are not affected). */
gpe_status gpe_batch_destroy(gpe_batch batch);
gpe_status gpe_batch_work_bytes(gpe_batch batch, gpe_dtype dtype, int32_t mode, int64_t nsteps,
                                int64_t ckpt_every, size_t* bytes);

/* Real time for every instance: instance i uses ramps[i] (RF_RAMP, with
 * field = its U) and params[i] (g, dt); all instances take nsteps steps from
 * t0 with the same integrator (params[i].integrator equal for all i).  use_graph != 0 captures one step (all stage kernels of all instances)
 * into a hipGraph on first use and replays it; the step counter lives in
 * device memory so one graph serves every step.  final_host: optional n
 * observations (per-instance FP64 reductions). */
gpe_status gpe_batch_real_time(gpe_batch batch, gpe_dtype dtype, void* psi, const void* field,
                               const gpe_ramp* ramps, const gpe_params* params, double t0, int64_t nsteps,
                               int32_t use_graph, void* work, size_t work_bytes, void* stream,
                               gpe_obs* final_host);

/* Batched gpe_fidelity_grad: loss_host[n], grad_host[n x GPE_MAX_KNOTS]
 * (instance i's gradient at grad_host + i*GPE_MAX_KNOTS, n_knots entries).
 * use_graph != 0: the forward sweep replays the captured step graph of
 * gpe_batch_real_time (checkpoint copies are enqueued between replays); the
 * reverse sweep is launched eagerly. */
gpe_status gpe_batch_fidelity_grad(gpe_batch batch, gpe_dtype dtype, const void* psi0, const void* psi_target,
                                   const void* field, const gpe_ramp* ramps, const gpe_params* params,
                                   double t0, int64_t nsteps, int64_t ckpt_every, int32_t use_graph,
                                   void* work, size_t work_bytes, void* stream, double* loss_host,
                                   double* grad_host);

/* ---- Launch configuration and autotuning -----------------------------
 * A launch configuration is an index into the table of compiled kernel
 * variants: workgroup size (64 to 1024 lanes) x sites per lane (1 to 8), the
 * order in which chunks are
 * handed to the XCDs (0 array order, 1 contiguous eighths, 2/3 blocks of
 * 64/256 chunks dealt round-robin, 4 the x-th eighth of every x-plane's
 * chunks to XCD x, plane after plane), and the
 * RK4 storage scheme (0: the App. A form, whose last stage reads y0, y2, y3;
 * 1: the second stage also stores A = (-y0 + y2 + 2 y3)/3 so the last stage
 * reads A alone, 16 fewer bytes per site per complex128 step; both give the
 * RK4 result up to rounding), whether streams touched once per pass use
 * non-temporal loads/stores, and whether the chunk's stencil input is staged
 * in LDS (1: the k-1 / k+1 and in-window j-1 / j+1 neighbours come from LDS;
 * 0: every neighbour is loaded from global memory and the pass has one
 * workgroup barrier fewer).  Every variant computes the same stencil
 * arithmetic; results differ only by the rounding of the FP64 reductions,
 * whose grouping follows the chunk size, and of the RK4 storage scheme.
 * gpe_config_count/gpe_config_describe list
 * them; variant 0 is the default.  The grid's (or batch's) configuration is
 * used by every later call on it. */
int32_t gpe_config_count(void);
gpe_status gpe_config_describe(int32_t config, int32_t* block, int32_t* sites_per_lane, int32_t* xcd_map,
                               int32_t* rk_scheme, int32_t* nontemporal, int32_t* lds_stage);
gpe_status gpe_grid_set_config(gpe_grid grid, int32_t config);
gpe_status gpe_grid_get_config(gpe_grid grid, int32_t* config);
gpe_status gpe_batch_set_config(gpe_batch batch, int32_t config);
gpe_status gpe_batch_get_config(gpe_batch batch, int32_t* config);

/* Time every configuration on `reps` steps of psi of one phase (contents
 * are advanced; pass a scratch copy), in three interleaved rounds keeping
 * each variant's fastest, select the fastest and store it on the grid.
 *   mode: GPE_MODE_RT (real time with params.integrator; work sized for it),
 *         GPE_MODE_ITP or GPE_MODE_ITP_REAL (imaginary time on a complex /
 *         real state; params.integrator must be 0).
 *   times_ms_host: optional gpe_config_count() doubles (ms per step). */
gpe_status gpe_grid_autotune(gpe_grid grid, gpe_dtype dtype, int32_t mode, void* psi, const gpe_potential* pot,
                             const gpe_params* params, int32_t reps, void* work, size_t work_bytes,
                             void* stream, int32_t* best_config, double* times_ms_host);

/* Every gpe_grid_autotune result is also recorded in a process-wide cache
 * keyed by (dtype, mode, floor(log2 n_active), floor(log2 mean segment
 * length)).  gpe_grid_apply_tuned gives the grid the cached configuration of
 * its class for that phase (*config = that index) or leaves it unchanged
 * (*config = -1 when the class has not been tuned).  gpe_autotune_cache_clear
 * empties the cache.  The cache is guarded by a lock. */
gpe_status gpe_grid_apply_tuned(gpe_grid grid, gpe_dtype dtype, int32_t mode, int32_t* config);
gpe_status gpe_autotune_cache_clear(void);

/* Batched ramp sweeps (the Sec. V ramp-optimisation workload, many ramps per
 * launch): time every configuration on `reps` real-time steps of the whole
 * batch (the launches of gpe_batch_real_time with the same ramps, params and
 * use_graph; psi is advanced, pass a scratch copy), three interleaved rounds
 * keeping each variant's fastest, select the fastest and store it on the
 * batch.  With use_graph each variant's step graph is captured in an untimed
 * first step, so replays are what is timed.  The result is cached like
 * gpe_grid_autotune's, keyed by (dtype, floor(log2 total active sites),
 * floor(log2 mean segment length), floor(log2 instance count));
 * gpe_batch_apply_tuned gives a batch of the same class the cached
 * configuration (*config = -1 when none).
 *   work: >= gpe_batch_work_bytes(.., GPE_MODE_RT (or the integrator's mode), ..).
 *   times_ms_host: optional gpe_config_count() doubles (ms per step). */
gpe_status gpe_batch_autotune(gpe_batch batch, gpe_dtype dtype, void* psi, const void* field, const gpe_ramp* ramps,
                              const gpe_params* params, int32_t reps, int32_t use_graph, void* work,
                              size_t work_bytes, void* stream, int32_t* best_config, double* times_ms_host);
gpe_status gpe_batch_apply_tuned(gpe_batch batch, gpe_dtype dtype, int32_t* config);

/* ---- Per-kernel timing -----------------------------------------------
 * When enabled, every kernel launch of the library is bracketed by HIP
 * events on its stream and the elapsed time is accumulated per kernel
 * family (names from gpe_timing_name).  Reading the totals synchronises. */
gpe_status gpe_timing_enable(int32_t enable);
gpe_status gpe_timing_reset(void);
int32_t gpe_timing_count(void);
const char* gpe_timing_name(int32_t family);
gpe_status gpe_timing_read(int32_t family, int64_t* launches, double* total_ms);

/* A plain streaming copy of `bytes` bytes from src to dst (device buffers,
 * 16-byte aligned, not overlapping; bytes a multiple of 16): one 16-byte
 * load and one 16-byte store per lane and nothing else.  It measures the
 * achievable HBM bandwidth that the passes' roofline is read against (timing
 * family "stream_copy").  Stream-ordered.  GPE_ERR_ARG for a NULL or
 * misaligned pointer, a size that is not a multiple of 16 or needs more than
 * 2^31 - 1 workgroups, or overlapping buffers. */
gpe_status gpe_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* GPE_H */
