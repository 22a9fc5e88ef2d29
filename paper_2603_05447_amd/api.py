"""Python binding of the C ABI: argument marshalling only.

Device memory and streams come from PyTorch (ROCm); every step of the solver
runs in the HIP kernels of libgpe.so.  There is no CPU fallback: if the
library is missing, importing this module's functions raises.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from ._lib import check

_CDT = {torch.complex128: L.GPE_C128, torch.complex64: L.GPE_C64}
_RDT = {L.GPE_C128: torch.float64, L.GPE_C64: torch.float32}
# real states (imaginary time from a real start): float64 pairs with GPE_C128
_RSTATE = {torch.float64: L.GPE_C128, torch.float32: L.GPE_C64}


def _stream(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _used_on(t: torch.Tensor, stream) -> torch.Tensor:
    """Tell torch's caching allocator that `t` is used on `stream` (a torch
    stream other than the current one), so its memory is not handed out again
    before the work queued there has finished."""
    if stream is not None and isinstance(stream, torch.cuda.Stream) and stream != torch.cuda.current_stream():
        t.record_stream(stream)
    return t


def _dtype_of(psi: torch.Tensor) -> int:
    if psi.dtype not in _CDT:
        raise TypeError("psi must be complex128 or complex64")
    if not psi.is_cuda or not psi.is_contiguous():
        raise ValueError("psi must be a contiguous CUDA/HIP tensor")
    return _CDT[psi.dtype]


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _dbl(a) -> C.Array:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return (C.c_double * a.size)(*a.tolist())


class Potential:
    """Static V(x), RF-dressed ramp V = sqrt((U - Delta(t))^2 + omega^2), or
    one stage of a staged ramp V = (1 - l) V_a + l V_b (LERP)."""

    def __init__(self, kind: int, field: torch.Tensor, omega: float = 0.0, knot_t=None, knot_delta=None,
                 field2: Optional[torch.Tensor] = None):
        self.kind = kind
        self.field = field
        self.field2 = field2
        self.omega = float(omega)
        self.knot_t = None if knot_t is None else np.asarray(knot_t, np.float64)
        self.knot_delta = None if knot_delta is None else np.asarray(knot_delta, np.float64)

    @staticmethod
    def static(V: torch.Tensor) -> "Potential":
        return Potential(L.GPE_POT_STATIC, V)

    @staticmethod
    def rf(U: torch.Tensor, omega: float, knot_t, knot_delta) -> "Potential":
        return Potential(L.GPE_POT_RF_RAMP, U, omega, knot_t, knot_delta)

    @staticmethod
    def shell(r: torch.Tensor, lam: float, knot_t, knot_radius) -> "Potential":
        """Harmonic shell lam/2 (r - R0(t))^2 around the per-site distances r,
        with the radius R0(t) ramped through (knot_t, knot_radius)."""
        return Potential(L.GPE_POT_SHELL_RAMP, r, lam, knot_t, knot_radius)

    @staticmethod
    def lerp(Va: torch.Tensor, Vb: torch.Tensor, t_a: float, t_b: float) -> "Potential":
        """Stage potential interpolated linearly in time from Va (at t_a) to Vb (at t_b)."""
        return Potential(L.GPE_POT_LERP, Va, 0.0, [t_a, t_b], None, field2=Vb)

    def with_knots(self, knot_delta) -> "Potential":
        return Potential(self.kind, self.field, self.omega, self.knot_t, knot_delta)

    def as_c(self, dtype: int):
        want = _RDT[dtype]
        if self.field.dtype != want or not self.field.is_cuda or not self.field.is_contiguous():
            raise TypeError(f"potential field must be a contiguous CUDA tensor of {want}")
        p = L.Potential()
        p.kind = self.kind
        p.field = self.field.data_ptr()
        p.omega = self.omega
        keep = []
        if self.kind in (L.GPE_POT_RF_RAMP, L.GPE_POT_SHELL_RAMP):
            kt, kd = _dbl(self.knot_t), _dbl(self.knot_delta)
            keep = [kt, kd]
            p.n_knots = len(self.knot_t)
            p.knot_t = C.cast(kt, C.POINTER(C.c_double))
            p.knot_delta = C.cast(kd, C.POINTER(C.c_double))
        elif self.kind == L.GPE_POT_LERP:
            f2 = self.field2
            if f2 is None or f2.dtype != want or not f2.is_cuda or not f2.is_contiguous():
                raise TypeError(f"stage end field must be a contiguous CUDA tensor of {want}")
            kt = _dbl(self.knot_t)
            keep = [kt]
            p.n_knots = 2
            p.knot_t = C.cast(kt, C.POINTER(C.c_double))
            p.field2 = f2.data_ptr()
        else:
            p.n_knots = 0
        return p, keep


INTEGRATORS = {"rk4": L.GPE_RK4, "rkhe3": L.GPE_RKHE3, "rkck": L.GPE_RKCK}
_RT_MODE = {L.GPE_RK4: L.GPE_MODE_RT, L.GPE_RKHE3: L.GPE_MODE_RT_RKHE3, L.GPE_RKCK: L.GPE_MODE_RT_RKCK}
_TUNE_MODE = {"rt": L.GPE_MODE_RT, "itp": L.GPE_MODE_ITP, "itp_real": L.GPE_MODE_ITP_REAL}


def _integrator(name: str) -> int:
    if name not in INTEGRATORS:
        raise ValueError(f"integrator must be one of {sorted(INTEGRATORS)}, got {name!r}")
    return INTEGRATORS[name]


def make_params(g: float, dt: float, norm_target: float = 1.0, obs_every: int = 0, check_stability: bool = True,
                integrator: str = "rk4"):
    p = L.Params()
    p.g, p.dt, p.norm_target = float(g), float(dt), float(norm_target)
    p.obs_every = int(obs_every)
    p.skip_stability_check = 0 if check_stability else 1
    p.integrator = _integrator(integrator)
    return p


def _obs_dict(o: L.Obs) -> dict:
    return {"norm": o.norm, "energy": o.energy, "mu": o.mu}


class Grid:
    """Compact layout of one masked grid (gpe_grid)."""

    def __init__(self, n, h, x0, runs=None, mask=None, device: int = 0):
        lib = L.load()
        geom = L.Geometry()
        for d in range(3):
            geom.n[d], geom.h[d], geom.x0[d] = int(n[d]), float(h[d]), float(x0[d])
        handle = C.c_void_p()
        if runs is not None:
            r = np.ascontiguousarray(np.asarray(runs, dtype=np.int64))
            check(lib.gpe_grid_create_runs(C.byref(geom), r.shape[0], r.ctypes.data, int(device), C.byref(handle)))
        elif mask is not None:
            m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
            check(lib.gpe_grid_create(C.byref(geom), m.ctypes.data, int(device), C.byref(handle)))
        else:
            raise ValueError("need runs or mask")
        self._h = handle
        self.device = int(device)
        self.x0 = tuple(float(v) for v in x0)
        self.n = tuple(int(v) for v in n)
        self.h = tuple(float(v) for v in h)
        self.dV = self.h[0] * self.h[1] * self.h[2]
        na, nr, ns = C.c_int64(), C.c_int64(), C.c_int64()
        check(lib.gpe_grid_info(handle, C.byref(na), C.byref(nr), C.byref(ns)))
        self.n_active, self.n_runs, self.n_segments = na.value, nr.value, ns.value
        self._work = {}

    @staticmethod
    def from_box(box, runs=None, mask=None, device: int = 0) -> "Grid":
        return Grid(box.n, box.h, box.x0, runs=runs, mask=mask, device=device)

    @staticmethod
    def from_threshold(n, h, x0, Va_box: torch.Tensor, Vb_box: Optional[torch.Tensor], cutoff: float,
                       device: int = 0) -> "Grid":
        """Post-selection on the device: keep the box points where
        min(Va_box, Vb_box) < cutoff (gpe_grid_create_threshold)."""
        dt_ = {torch.float64: L.GPE_C128, torch.float32: L.GPE_C64}.get(Va_box.dtype)
        if dt_ is None:
            raise TypeError("Va_box must be float64 or float32")
        for t in (Va_box, Vb_box):
            if t is not None and (t.dtype != Va_box.dtype or not t.is_cuda or not t.is_contiguous()
                                  or t.numel() != int(n[0]) * int(n[1]) * int(n[2])):
                raise ValueError("potentials must be contiguous CUDA box arrays of one real dtype")
        geom = L.Geometry()
        for d in range(3):
            geom.n[d], geom.h[d], geom.x0[d] = int(n[d]), float(h[d]), float(x0[d])
        handle = C.c_void_p()
        check(L.load().gpe_grid_create_threshold(C.byref(geom), dt_, Va_box.data_ptr(), _ptr(Vb_box),
                                                  float(cutoff), int(device), C.byref(handle)))
        return Grid._wrap(handle, n, h, x0, int(device))

    @staticmethod
    def _wrap(handle, n, h, x0, device: int) -> "Grid":
        g = Grid.__new__(Grid)
        g._h = handle
        g.device = device
        g.x0 = tuple(float(v) for v in x0)
        g.n = tuple(int(v) for v in n)
        g.h = tuple(float(v) for v in h)
        g.dV = g.h[0] * g.h[1] * g.h[2]
        na, nr, ns = C.c_int64(), C.c_int64(), C.c_int64()
        check(L.load().gpe_grid_info(handle, C.byref(na), C.byref(nr), C.byref(ns)))
        g.n_active, g.n_runs, g.n_segments = na.value, nr.value, ns.value
        g._work = {}
        return g

    def remap_from(self, src: "Grid", psi_src: torch.Tensor, out: Optional[torch.Tensor] = None,
                   stream=None) -> torch.Tensor:
        """psi on this grid from psi on `src` (same box): common sites copied,
        new sites zero (gpe_remap)."""
        dt_ = _dtype_of(psi_src)
        if psi_src.numel() != src.n_active:
            raise ValueError("psi_src must hold the source grid's n_active values")
        if out is None:
            out = torch.empty(self.n_active, dtype=psi_src.dtype, device=psi_src.device)
        if out.numel() != self.n_active or out.dtype != psi_src.dtype or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor of this grid's n_active values")
        check(L.load().gpe_remap(src._h, self._h, dt_, psi_src.data_ptr(), out.data_ptr(), _stream(stream)))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                L.load().gpe_grid_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h

    # ---- host tables ----------------------------------------------------
    def segments(self) -> np.ndarray:
        out = np.zeros((self.n_segments, 8), np.int32)
        check(L.load().gpe_grid_segments(self._h, out.ctypes.data))
        return out

    def runs(self) -> np.ndarray:
        out = np.zeros((self.n_runs, 5), np.int64)
        check(L.load().gpe_grid_runs(self._h, out.ctypes.data))
        return out

    def apply_tuned(self, dtype: int, phase: str = "rt") -> Optional[int]:
        """Take the launch configuration autotuned for this grid's size /
        segment-length class and phase (any grid of the process), if there
        is one."""
        c = C.c_int32()
        check(L.load().gpe_grid_apply_tuned(self._h, int(dtype), _TUNE_MODE[phase], C.byref(c)))
        return None if c.value < 0 else c.value

    def set_stencil(self, points: int) -> None:
        """7-point (default), 19-point HOC (App. B eq. (B2)) or 27-point cubic Laplacian."""
        check(L.load().gpe_grid_set_stencil(self._h, int(points)))

    def get_stencil(self) -> int:
        c = C.c_int32()
        check(L.load().gpe_grid_get_stencil(self._h, C.byref(c)))
        return c.value

    def hoc_segments(self, points: int = 19) -> np.ndarray:
        """The 19- or 27-point segment table: rows {start, length, flags, off[T], 0}."""
        n = C.c_int64()
        check(L.load().gpe_grid_stencil_segments(self._h, int(points), C.byref(n), None))
        out = np.zeros((n.value, 4 + (16 if points == 19 else 24)), np.int32)
        check(L.load().gpe_grid_stencil_segments(self._h, int(points), C.byref(n), out.ctypes.data))
        return out

    # ---- work buffers ---------------------------------------------------
    def work_bytes(self, dtype: int, mode: int, nsteps: int = 0, ckpt_every: int = 0) -> int:
        b = C.c_size_t()
        check(L.load().gpe_work_bytes(self._h, dtype, mode, int(nsteps), int(ckpt_every), C.byref(b)))
        return b.value

    def work(self, dtype: int, mode: int, nsteps: int = 0, ckpt_every: int = 0) -> torch.Tensor:
        nb = self.work_bytes(dtype, mode, nsteps, ckpt_every)
        key = (dtype, mode)
        w = self._work.get(key)
        if w is None or w.numel() < nb:
            w = torch.empty(max(nb, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
            self._work[key] = w
        return w

    def release_work(self):
        self._work.clear()

    # ---- solver calls ---------------------------------------------------
    def imag_time(self, psi: torch.Tensor, pot: Potential, g: float, dt: float, steps: int,
                  norm_target: float = 1.0, obs_every: int = 0, history: Optional[torch.Tensor] = None,
                  stream=None, observe: bool = True, check_stability: bool = True) -> Optional[dict]:
        """Imaginary time in place.  A complex psi (complex128/complex64) runs
        gpe_imag_time; a real psi (float64/float32) runs gpe_imag_time_real."""
        real = psi.dtype in _RSTATE
        if real:
            if not psi.is_cuda or not psi.is_contiguous():
                raise ValueError("psi must be a contiguous CUDA/HIP tensor")
            dt_ = _RSTATE[psi.dtype]
        else:
            dt_ = _dtype_of(psi)
        cp, keep = pot.as_c(dt_)
        prm = make_params(g, dt, norm_target, obs_every, check_stability)
        w = _used_on(self.work(dt_, L.GPE_MODE_ITP_REAL if real else L.GPE_MODE_ITP, steps), stream)
        o = L.Obs()
        fn = L.load().gpe_imag_time_real if real else L.load().gpe_imag_time
        check(fn(self._h, dt_, psi.data_ptr(), C.byref(cp), C.byref(prm), int(steps), w.data_ptr(), w.numel(),
                 _stream(stream), C.byref(o) if observe else None, _ptr(history)))
        return _obs_dict(o) if observe else None

    def real_time(self, psi: torch.Tensor, pot: Potential, g: float, dt: float, steps: int, t0: float = 0.0,
                  obs_every: int = 0, history: Optional[torch.Tensor] = None, stream=None, observe: bool = True,
                  check_stability: bool = True, integrator: str = "rk4") -> Optional[dict]:
        dt_ = _dtype_of(psi)
        cp, keep = pot.as_c(dt_)
        prm = make_params(g, dt, 1.0, obs_every, check_stability, integrator)
        w = _used_on(self.work(dt_, _RT_MODE[prm.integrator], steps), stream)
        o = L.Obs()
        check(L.load().gpe_real_time(self._h, dt_, psi.data_ptr(), C.byref(cp), C.byref(prm), float(t0),
                                     int(steps), w.data_ptr(), w.numel(), _stream(stream),
                                     C.byref(o) if observe else None, _ptr(history)))
        return _obs_dict(o) if observe else None

    def observe(self, psi: torch.Tensor, pot: Potential, t: float, g: float, stream=None) -> dict:
        dt_ = _dtype_of(psi)
        cp, keep = pot.as_c(dt_)
        o = L.Obs()
        check(L.load().gpe_observe(self._h, dt_, psi.data_ptr(), C.byref(cp), float(t), float(g), _stream(stream),
                                   C.byref(o)))
        return _obs_dict(o)

    def overlap(self, a: torch.Tensor, b: torch.Tensor, stream=None) -> complex:
        dt_ = _dtype_of(a)
        if b.dtype != a.dtype:
            raise TypeError("a and b must have the same dtype")
        out = (C.c_double * 2)()
        check(L.load().gpe_overlap(self._h, dt_, a.data_ptr(), b.data_ptr(), _stream(stream), out))
        return complex(out[0], out[1])

    def fidelity_grad(self, psi0: torch.Tensor, target: torch.Tensor, pot: Potential, g: float, dt: float,
                      steps: int, t0: float = 0.0, ckpt_every: int = 0, psi_final: Optional[torch.Tensor] = None,
                      stream=None, check_stability: bool = True):
        dt_ = _dtype_of(psi0)
        cp, keep = pot.as_c(dt_)
        prm = make_params(g, dt, 1.0, 0, check_stability)
        nb = self.work_bytes(dt_, L.GPE_MODE_ADJ, steps, ckpt_every)
        w = _used_on(torch.empty(max(nb, 256), dtype=torch.uint8, device=psi0.device), stream)
        loss = C.c_double()
        grad = (C.c_double * L.GPE_MAX_KNOTS)()
        check(L.load().gpe_fidelity_grad(self._h, dt_, psi0.data_ptr(), target.data_ptr(), C.byref(cp),
                                         C.byref(prm), float(t0), int(steps), int(ckpt_every), w.data_ptr(),
                                         w.numel(), _stream(stream), C.byref(loss), grad, _ptr(psi_final)))
        n = len(pot.knot_t)
        return loss.value, np.array(grad[:n])

    def pack(self, box: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Box array -> compact.  Complex (psi) or real (a potential field)."""
        nbox = self.n[0] * self.n[1] * self.n[2]
        if box.numel() != nbox:
            raise ValueError(f"box array has {box.numel()} elements, the grid's box {nbox}")
        real = box.dtype in _RSTATE
        if real:
            if not box.is_cuda or not box.is_contiguous():
                raise ValueError("box must be a contiguous CUDA/HIP tensor")
            dt_ = _RSTATE[box.dtype]
        else:
            dt_ = _dtype_of(box)
        if out is None:
            out = torch.empty(self.n_active, dtype=box.dtype, device=box.device)
        if out.numel() != self.n_active or out.dtype != box.dtype or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor of n_active elements of the box's dtype")
        fn = L.load().gpe_pack_real if real else L.load().gpe_pack
        check(fn(self._h, dt_, box.data_ptr(), out.data_ptr(), _stream(stream)))
        return out

    def unpack(self, compact: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        dt_ = _dtype_of(compact)
        if compact.numel() != self.n_active:
            raise ValueError("compact array must hold n_active elements")
        if out is None:
            out = torch.empty(self.n, dtype=compact.dtype, device=compact.device)
        if out.numel() != self.n[0] * self.n[1] * self.n[2]:
            raise ValueError("out must hold the whole box")
        check(L.load().gpe_unpack(self._h, dt_, compact.data_ptr(), out.data_ptr(), _stream(stream)))
        return out

    # ---- launch configuration -------------------------------------------
    def set_config(self, config: int) -> None:
        check(L.load().gpe_grid_set_config(self._h, int(config)))

    def get_config(self) -> int:
        c = C.c_int32()
        check(L.load().gpe_grid_get_config(self._h, C.byref(c)))
        return c.value

    def autotune(self, psi: torch.Tensor, pot: Potential, g: float, dt: float, reps: int = 5, stream=None,
                 integrator: str = "rk4", phase: str = "rt"):
        """Time every launch variant on `reps` steps of one phase ("rt": real
        time with `integrator`; "itp": imaginary time, on a real state when
        psi is real) and keep the fastest.  psi is advanced."""
        real = psi.dtype in _RSTATE
        if real and phase != "itp":
            raise ValueError("a real state tunes imaginary time only (phase='itp')")
        if real:
            if not psi.is_cuda or not psi.is_contiguous():
                raise ValueError("psi must be a contiguous CUDA/HIP tensor")
            dt_ = _RSTATE[psi.dtype]
        else:
            dt_ = _dtype_of(psi)
        cp, keep = pot.as_c(dt_)
        if phase == "itp":
            mode = L.GPE_MODE_ITP_REAL if real else L.GPE_MODE_ITP
            prm = make_params(g, dt)
            w = _used_on(self.work(dt_, mode, reps), stream)
        elif phase == "rt":
            prm = make_params(g, dt, integrator=integrator)
            mode = L.GPE_MODE_RT
            w = _used_on(self.work(dt_, _RT_MODE[prm.integrator], reps), stream)
        else:
            raise ValueError("phase must be 'rt' or 'itp'")
        n = config_count()
        times = (C.c_double * n)(*([-1.0] * n))
        best = C.c_int32()
        check(L.load().gpe_grid_autotune(self._h, dt_, mode, psi.data_ptr(), C.byref(cp), C.byref(prm), int(reps),
                                         w.data_ptr(), w.numel(), _stream(stream), C.byref(best), times))
        return best.value, list(times)


class Batch:
    """Several grids concatenated into one compact layout (gpe_batch)."""

    def __init__(self, grids: Sequence[Grid], device: int = 0):
        lib = L.load()
        arr = (C.c_void_p * len(grids))(*[g.handle.value for g in grids])
        h = C.c_void_p()
        check(lib.gpe_batch_create(len(grids), arr, int(device), C.byref(h)))
        self._h = h
        self.grids = list(grids)
        self.device = int(device)
        off = (C.c_int64 * (len(grids) + 1))()
        check(lib.gpe_batch_offsets(h, off))
        self.offsets = np.array(off[:], dtype=np.int64)
        self.total = int(self.offsets[-1])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                L.load().gpe_batch_destroy(h)
            except Exception:
                pass
            self._h = None

    def work_bytes(self, dtype: int, mode: int, nsteps: int = 0, ckpt_every: int = 0) -> int:
        b = C.c_size_t()
        check(L.load().gpe_batch_work_bytes(self._h, dtype, mode, int(nsteps), int(ckpt_every), C.byref(b)))
        return b.value

    def set_config(self, config: int) -> None:
        check(L.load().gpe_batch_set_config(self._h, int(config)))

    def get_config(self) -> int:
        c = C.c_int32()
        check(L.load().gpe_batch_get_config(self._h, C.byref(c)))
        return c.value

    def autotune(self, psi: torch.Tensor, field: torch.Tensor, ramps, gs, dts, reps: int = 3,
                 use_graph: bool = True, stream=None, integrator: str = "rk4"):
        """Time every launch variant on `reps` real-time steps of the whole
        batch (gpe_batch_autotune) and keep the fastest; psi is advanced.
        Returns (best variant, ms per step of every variant)."""
        dt_ = _dtype_of(psi)
        ra, keep = self._ramps(ramps)
        pa = self._params(gs, dts, integrator)
        nb = self.work_bytes(dt_, _RT_MODE[pa[0].integrator], reps)
        w = _used_on(torch.empty(max(nb, 256), dtype=torch.uint8, device=psi.device), stream)
        n = config_count()
        times = (C.c_double * n)(*([-1.0] * n))
        best = C.c_int32()
        check(L.load().gpe_batch_autotune(self._h, dt_, psi.data_ptr(), field.data_ptr(), ra, pa, int(reps),
                                          1 if use_graph else 0, w.data_ptr(), w.numel(), _stream(stream),
                                          C.byref(best), times))
        return best.value, list(times)

    def apply_tuned(self, dtype: int) -> Optional[int]:
        """Take the launch configuration autotuned for this batch's class, if any."""
        c = C.c_int32()
        check(L.load().gpe_batch_apply_tuned(self._h, int(dtype), C.byref(c)))
        return None if c.value < 0 else c.value

    @staticmethod
    def _ramps(ramps):
        """ramps[i] = (omega, knot_t, knot_values) for an RF ramp, or
        (omega, knot_t, knot_values, kind) with kind GPE_POT_RF_RAMP or
        GPE_POT_SHELL_RAMP."""
        n = len(ramps)
        arr = (L.Ramp * n)()
        keep = []
        for i, rp in enumerate(ramps):
            omega, kt, kd = rp[:3]
            a, b = _dbl(kt), _dbl(kd)
            keep += [a, b]
            arr[i].omega = float(omega)
            arr[i].n_knots = len(kt)
            arr[i].kind = int(rp[3]) if len(rp) > 3 else L.GPE_POT_RF_RAMP
            arr[i].knot_t = C.cast(a, C.POINTER(C.c_double))
            arr[i].knot_delta = C.cast(b, C.POINTER(C.c_double))
        return arr, keep

    @staticmethod
    def _params(gs, dts, integrator: str = "rk4", check_stability: bool = True):
        arr = (L.Params * len(gs))()
        for i, (g, dt) in enumerate(zip(gs, dts)):
            arr[i] = make_params(g, dt, integrator=integrator, check_stability=check_stability)
        return arr

    def real_time(self, psi: torch.Tensor, field: torch.Tensor, ramps, gs, dts, steps: int, t0: float = 0.0,
                  use_graph: bool = True, work: Optional[torch.Tensor] = None, stream=None, observe: bool = True,
                  integrator: str = "rk4", check_stability: bool = True):
        dt_ = _dtype_of(psi)
        ra, keep = self._ramps(ramps)
        pa = self._params(gs, dts, integrator, check_stability)
        nb = self.work_bytes(dt_, _RT_MODE[pa[0].integrator], steps)
        if work is None or work.numel() < nb:
            work = torch.empty(max(nb, 256), dtype=torch.uint8, device=psi.device)
        _used_on(work, stream)
        obs = (L.Obs * len(self.grids))()
        check(L.load().gpe_batch_real_time(self._h, dt_, psi.data_ptr(), field.data_ptr(), ra, pa, float(t0),
                                           int(steps), 1 if use_graph else 0, work.data_ptr(), work.numel(),
                                           _stream(stream), obs if observe else None))
        return [_obs_dict(o) for o in obs] if observe else None

    def fidelity_grad(self, psi0: torch.Tensor, target: torch.Tensor, field: torch.Tensor, ramps, gs, dts,
                      steps: int, t0: float = 0.0, ckpt_every: int = 0, use_graph: bool = False, stream=None,
                      check_stability: bool = True):
        dt_ = _dtype_of(psi0)
        ra, keep = self._ramps(ramps)
        pa = self._params(gs, dts, check_stability=check_stability)
        nb = self.work_bytes(dt_, L.GPE_MODE_ADJ, steps, ckpt_every)
        w = _used_on(torch.empty(max(nb, 256), dtype=torch.uint8, device=psi0.device), stream)
        n = len(self.grids)
        loss = (C.c_double * n)()
        grad = (C.c_double * (n * L.GPE_MAX_KNOTS))()
        check(L.load().gpe_batch_fidelity_grad(self._h, dt_, psi0.data_ptr(), target.data_ptr(), field.data_ptr(),
                                               ra, pa, float(t0), int(steps), int(ckpt_every),
                                               1 if use_graph else 0, w.data_ptr(),
                                               w.numel(), _stream(stream), loss, grad))
        g = np.array(grad[:], dtype=np.float64).reshape(n, L.GPE_MAX_KNOTS)
        return np.array(loss[:]), [g[i, :len(ramps[i][1])] for i in range(n)]


class FidelityGrad(torch.autograd.Function):
    """loss = 1 - |<target|psi(T)>|^2 as a differentiable function of the ramp
    knot values; forward runs the RK4 forward sweep and the adjoint sweep on
    the device (one ABI call) and caches dL/dknots for backward."""

    @staticmethod
    def forward(ctx, knots: torch.Tensor, grid: Grid, psi0: torch.Tensor, target: torch.Tensor, U: torch.Tensor,
                omega: float, knot_t, g: float, dt: float, steps: int, ckpt_every: int = 0,
                kind: int = L.GPE_POT_RF_RAMP):
        kd = knots.detach().to("cpu", torch.float64).numpy()
        pot = Potential(kind, U, omega, knot_t, kd)
        loss, grad = grid.fidelity_grad(psi0, target, pot, g, dt, steps, 0.0, ckpt_every)
        ctx.save_for_backward(torch.as_tensor(grad, dtype=knots.dtype, device=knots.device))
        return torch.tensor(loss, dtype=knots.dtype, device=knots.device)

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return (grad_out * grad,) + (None,) * 11


class BatchFidelityGrad(torch.autograd.Function):
    """Per-instance losses 1 - |<target_i|psi_i(T)>|^2 of a batch as a
    differentiable function of a (n_instances, n_knots) tensor of knot values
    (all instances share one knot count); one ABI call runs the batched
    forward and adjoint sweeps and the gradients are cached for backward."""

    @staticmethod
    def forward(ctx, knots: torch.Tensor, batch: "Batch", psi0: torch.Tensor, target: torch.Tensor,
                field: torch.Tensor, omegas, knot_ts, gs, dts, steps: int, ckpt_every: int = 0,
                use_graph: bool = False, kinds=None):
        kd = knots.detach().to("cpu", torch.float64).numpy()
        if kd.ndim != 2 or kd.shape[0] != len(batch.grids):
            raise ValueError("knots must be (n_instances, n_knots)")
        ramps = [(omegas[i], knot_ts[i], kd[i], L.GPE_POT_RF_RAMP if kinds is None else kinds[i])
                 for i in range(kd.shape[0])]
        loss, grads = batch.fidelity_grad(psi0, target, field, ramps, gs, dts, steps, 0.0, ckpt_every,
                                          use_graph=use_graph)
        ctx.save_for_backward(torch.as_tensor(np.stack(grads), dtype=knots.dtype, device=knots.device))
        return torch.as_tensor(loss, dtype=knots.dtype, device=knots.device)

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return (grad_out[:, None] * grad,) + (None,) * 12


def stream_copy(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    """Plain streaming copy of src's bytes into dst on the device (the
    achievable-bandwidth reference kernel)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nb:
        raise ValueError("dst is smaller than src")
    check(L.load().gpe_stream_copy(src.data_ptr(), dst.data_ptr(), nb, _stream(stream)))


def config_count() -> int:
    return int(L.load().gpe_config_count())


def config_describe(i: int):
    b, s, x, r, nt, st = (C.c_int32() for _ in range(6))
    check(L.load().gpe_config_describe(int(i), C.byref(b), C.byref(s), C.byref(x), C.byref(r), C.byref(nt),
                                       C.byref(st)))
    return {"block": b.value, "sites_per_lane": s.value, "xcd_map": x.value, "rk_scheme": r.value,
            "nontemporal": nt.value, "lds_stage": st.value}


class KernelTimer:
    """Per-kernel-family HIP-event timing inside the library."""

    def __enter__(self):
        L.load().gpe_timing_reset()
        L.load().gpe_timing_enable(1)
        return self

    def __exit__(self, *exc):
        L.load().gpe_timing_enable(0)

    @staticmethod
    def read() -> dict:
        lib = L.load()
        out = {}
        for f in range(lib.gpe_timing_count()):
            n, ms = C.c_int64(), C.c_double()
            check(lib.gpe_timing_read(f, C.byref(n), C.byref(ms)))
            out[lib.gpe_timing_name(f).decode()] = {"launches": n.value, "total_ms": ms.value}
        return out


def staged_ramp(grid: Grid, psi: torch.Tensor, stage_fields: Sequence[torch.Tensor], mus: Sequence[float], g: float,
                dt: float, steps_per_stage: int, t0: float = 0.0, integrator: str = "rk4", stream=None,
                cutoff_factor: float = 0.0, check_stability: bool = True):
    """The staged ramp of Sec. V (gpe_staged_ramp_grids + gpe_staged_ramp_run).
    stage_fields[i] is the potential V_i on the whole box (device, real, box
    order); mus[i] the chemical potential of the ground state in V_i; psi
    lives on `grid`.  The library re-post-selects every stage's grid,
    carries psi over, and runs `steps_per_stage` real-time steps per stage
    with V interpolated linearly in time.  Returns the last stage's grid,
    psi on it and per-stage records."""
    lib = L.load()
    dt_ = _dtype_of(psi)
    if len(mus) != len(stage_fields):
        raise ValueError("one chemical potential per stage potential")
    if psi.numel() != grid.n_active:
        raise ValueError("psi must hold the grid's n_active values")
    want = _RDT[dt_]
    for f in stage_fields:
        if f.dtype != want or not f.is_cuda or not f.is_contiguous():
            raise TypeError(f"stage potentials must be contiguous CUDA tensors of {want}")
    S = len(stage_fields) - 1
    geom = L.Geometry()
    for d in range(3):
        geom.n[d], geom.h[d], geom.x0[d] = grid.n[d], grid.h[d], grid.x0[d]
    fields = (C.c_void_p * (S + 1))(*[f.data_ptr() for f in stage_fields])
    mu = _dbl(mus)
    handles = (C.c_void_p * S)()
    cuts = (C.c_double * S)()
    check(lib.gpe_staged_ramp_grids(C.byref(geom), dt_, S + 1, fields, mu, float(cutoff_factor), grid.device,
                                    handles, cuts))
    grids = [Grid._wrap(C.c_void_p(handles[i]), grid.n, grid.h, grid.x0, grid.device) for i in range(S)]
    psis = [_used_on(torch.empty(gr.n_active, dtype=psi.dtype, device=psi.device), stream) for gr in grids]
    prm = make_params(g, dt, integrator=integrator, check_stability=check_stability)
    nb = C.c_size_t()
    gh = (C.c_void_p * S)(*[gr.handle.value for gr in grids])
    check(lib.gpe_staged_ramp_work_bytes(S, gh, dt_, prm.integrator, C.byref(nb)))
    w = _used_on(torch.empty(max(nb.value, 256), dtype=torch.uint8, device=psi.device), stream)
    ps = (C.c_void_p * S)(*[p.data_ptr() for p in psis])
    rec = (C.c_double * (4 * S))()
    check(lib.gpe_staged_ramp_run(grid.handle, psi.data_ptr(), S, gh, ps, dt_, fields, C.byref(prm), float(t0),
                                  int(steps_per_stage), w.data_ptr(), w.numel(), _stream(stream), rec))
    records = [{"stage": i, "cutoff": cuts[i], "n_active": grids[i].n_active, "norm_after_remap": rec[4 * i],
                "norm_end": rec[4 * i + 1], "energy_end": rec[4 * i + 2], "mu_end": rec[4 * i + 3]}
               for i in range(S)]
    return grids[-1], psis[-1], records
