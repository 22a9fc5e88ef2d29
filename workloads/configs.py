"""The synthetic workloads (C1-C5) and small seeded test problems.

Each workload is a bounding box, an active-site run list, the per-site field
that defines its potential, and a seeded initial state.  The paper measures
on ab initio atom-chip RF-dressed potentials (Sec. V); those are not
available, so analytic shells of the same shape class stand in for them:

* a radial harmonic shell V = lambda/2 (r - R0)^2 (its radius R0 ramped in
  time for the batched sweep), and
* the RF-dressed form of eq. (10) written as V = sqrt((U - Delta)^2 + Omega^2)
  with a bare trap U = kappa/2 (x^2 + y^2 + 4 z^2).

The active set is {V < cutoff} (the Thomas-Fermi region of interest,
Sec. II.A), evaluated once here in float64 with a strict `<` and handed to
both the oracle and the HIP path.  For a time-dependent ramp the mask is the
union over the ramp, i.e. a bound on U.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .grids import (Box, complex_noise, normalise_input, runs_from_mask,
                    runs_from_predicate, site_coords)


@dataclass
class Workload:
    name: str
    box: Box
    runs: np.ndarray                 # (nruns, 4) int64: i, j, k0, k1
    field: np.ndarray                # per-site float64: V (static), U (RF form) or r (shell ramp)
    kind: str                        # "static", "rf" or "shell"
    omega: float = 0.0
    knot_t: Optional[np.ndarray] = None
    knot_delta: Optional[np.ndarray] = None
    g: float = 0.0
    dt: float = 1e-3
    steps: int = 1
    psi0: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)

    @property
    def n_active(self) -> int:
        return int(self.field.size)


# ----------------------------------------------------------------------------
# C1: 64^3 on [-8,8)^3, shell V = 20 (r-5)^2, mask V < 20, g = 100,
#     imaginary time 500 steps, dt = 1e-3, complex128.
# ----------------------------------------------------------------------------
def c1(seed: int = 0) -> Workload:
    box = Box.centred(64, 8.0)
    lam, R0 = 40.0, 5.0

    def active(x, y, z):
        r = np.sqrt(x * x + y * y + z * z)
        return 0.5 * lam * (r - R0) ** 2 < 20.0

    runs = runs_from_predicate(box, active)
    x, y, z = site_coords(box, runs)
    r = np.sqrt(x * x + y * y + z * z)
    V = 0.5 * lam * (r - R0) ** 2
    rng = np.random.default_rng(seed)
    psi = np.exp(-np.sqrt(lam) * (r - R0) ** 2 / 2.0) + complex_noise(rng, r.size, 1e-3)
    psi = normalise_input(psi, box.dV)
    return Workload("C1 shell 64^3 on [-8,8]^3, lambda=40 R0=5, mask V<20", box, runs, V, "static",
                    g=100.0, dt=1e-3, steps=500, psi0=psi)


# ----------------------------------------------------------------------------
# RF-dressed bubble family.
# ----------------------------------------------------------------------------
def _rf_runs(box: Box, kappa: float, u_lo: float, u_hi: float):
    def active(x, y, z):
        u = 0.5 * kappa * (x * x + y * y + 4.0 * z * z)
        return (u > u_lo) & (u < u_hi)
    return runs_from_predicate(box, active)


def _rf_U(box: Box, runs, kappa: float):
    x, y, z = site_coords(box, runs)
    return 0.5 * kappa * (x * x + y * y + 4.0 * z * z)


def rf_window(delta: float, omega: float, cutoff: float):
    """U-interval on which sqrt((U-delta)^2+omega^2) < cutoff."""
    w = np.sqrt(max(cutoff * cutoff - omega * omega, 0.0))
    return delta - w, delta + w


def tf_trial(V: np.ndarray, mu: float, g: float, dV: float, rng, noise: float) -> np.ndarray:
    """Thomas-Fermi trial state sqrt(max((mu - V)/g, 0)) plus seeded complex noise."""
    psi = np.sqrt(np.maximum((mu - V) / g, 0.0)).astype(np.complex128)
    psi = psi + complex_noise(rng, V.size, noise)
    return normalise_input(psi, dV)


# C2: 1024x1024x512, h = 0.0612, U = (x^2+y^2+4z^2)/2, Delta = 60, Omega = 2,
#     mask V < Omega + 25 = 27, g = 2000, dt = 2e-4.
def c2(seed: int = 1, box_n=(1024, 1024, 512), h: float = 0.0612) -> Workload:
    box = Box.centred(box_n, tuple(0.5 * n * h for n in box_n))
    delta, omega, cut = 60.0, 2.0, 27.0
    lo, hi = rf_window(delta, omega, cut)
    runs = _rf_runs(box, 1.0, lo, hi)
    U = _rf_U(box, runs, 1.0)
    V = np.sqrt((U - delta) ** 2 + omega ** 2)
    rng = np.random.default_rng(seed)
    psi = tf_trial(V, omega + 5.0, 2000.0, box.dV, rng, 1e-3)
    return Workload(f"C2 rf-bubble {box_n[0]}x{box_n[1]}x{box_n[2]} h={h}", box, runs, U, "rf",
                    omega=omega, knot_t=np.array([0.0]), knot_delta=np.array([delta]),
                    g=2000.0, dt=2e-4, steps=10000, psi0=psi,
                    extra={"itp_steps": 5000, "delta_itp": delta, "delta_rt": 62.0})


# C3: 256^3 on [-12.8,12.8)^3, Omega = 2, union mask over Delta in [-10, 40]
#     with cutoff 27, g = 1000, dt = 1e-3, T = 2, eight knots t_k = k T / 7.
def c3(box_n: int = 256, half_width: float = 12.8, steps: int = 2000, seed: int = 3) -> Workload:
    box = Box.centred(box_n, half_width)
    omega, cut = 2.0, 27.0
    d0, d1 = -10.0, 40.0
    lo, _ = rf_window(d0, omega, cut)
    _, hi = rf_window(d1, omega, cut)
    runs = _rf_runs(box, 1.0, lo, hi)
    U = _rf_U(box, runs, 1.0)
    dt = 1e-3 * 2000 / steps
    T = dt * steps
    kt = np.linspace(0.0, T, 8)
    kd = np.linspace(d0, d1, 8)
    rng = np.random.default_rng(seed)
    V0 = np.sqrt((U - d0) ** 2 + omega ** 2)
    psi = tf_trial(V0, np.min(V0) + 15.0, 1000.0, box.dV, rng, 1e-3)
    return Workload(f"C3 hollowing ramp {box_n}^3 h={box.h[0]:.4g}", box, runs, U, "rf", omega=omega,
                    knot_t=kt, knot_delta=kd, g=1000.0, dt=dt, steps=steps, psi0=psi)


# C4: 64 instances, cubic side n ~ U{96..192}, h = 0.1, rng(1000 + i):
#     harmonic shells V = lambda/2 (r - R0(t))^2 with lambda ~ U[20, 60] and the
#     radius R0 ramped linearly from 0.3 L to 0.6 L over 8 knots (field = r,
#     knot values = R0); the mask is the union over the ramp of V < 20, i.e.
#     r within sqrt(40 / lambda) of [0.3 L, 0.6 L]; g ~ U[100, 3000]; dt = 1e-3.
#     Start: the radial oscillator ground state of the first shell plus 1e-3
#     complex noise, normalised.
def c4_instance(i: int, n_lo: int = 96, n_hi: int = 192, h: float = 0.1, steps: int = 1000) -> Workload:
    rng = np.random.default_rng(1000 + i)
    n = int(rng.integers(n_lo, n_hi + 1))
    L = 0.5 * n * h
    lam = float(rng.uniform(20.0, 60.0))
    g = float(rng.uniform(100.0, 3000.0))
    r0, r1 = 0.3 * L, 0.6 * L
    wd = np.sqrt(2.0 * 20.0 / lam)
    box = Box.centred(n, L)

    def active(x, y, z):
        r = np.sqrt(x * x + y * y + z * z)
        return (r > r0 - wd) & (r < r1 + wd)

    runs = runs_from_predicate(box, active)
    x, y, z = site_coords(box, runs)
    r = np.sqrt(x * x + y * y + z * z)
    psi = np.exp(-np.sqrt(lam) * (r - r0) ** 2 / 2.0) + complex_noise(rng, r.size, 1e-3)
    psi = normalise_input(psi, box.dV)
    dt = 1e-3
    T = dt * steps
    return Workload(f"C4 instance {i} n={n}", box, runs, r, "shell", omega=lam,
                    knot_t=np.linspace(0.0, T, 8), knot_delta=np.linspace(r0, r1, 8),
                    g=g, dt=dt, steps=steps, psi0=psi)


# C5: 2048x2048x1024, h = 0.0306, kappa = 12.9, Delta = kappa/2 (0.92 Lx)^2,
#     Omega = 2, mask V < 61, g = 1e4, dt = 5e-5.
def c5(box_n=(2048, 2048, 1024), h: float = 0.0306, seed: int = 5) -> Workload:
    box = Box.centred(box_n, tuple(0.5 * n * h for n in box_n))
    kappa, omega, cut = 12.9, 2.0, 61.0
    Lx = 0.5 * box_n[0] * h
    delta = 0.5 * kappa * (0.92 * Lx) ** 2
    lo, hi = rf_window(delta, omega, cut)
    runs = _rf_runs(box, kappa, lo, hi)
    U = _rf_U(box, runs, kappa)
    V = np.sqrt((U - delta) ** 2 + omega ** 2)
    rng = np.random.default_rng(seed)
    psi = tf_trial(V, omega + 20.0, 1e4, box.dV, rng, 1e-3)
    return Workload(f"C5 thin shell {box_n[0]}x{box_n[1]}x{box_n[2]} h={h}", box, runs, U, "rf",
                    omega=omega, knot_t=np.array([0.0]), knot_delta=np.array([delta]),
                    g=1e4, dt=5e-5, steps=20000, psi0=psi)


# C5 subdomain: the large thin shell downscaled by `scale` in every direction
#     at the same spacing h, so the shell keeps its thickness in grid units:
#     the box side and the shell radius shrink by `scale`, kappa grows by it
#     (the same dU/dr at the shell, hence the same radial profile of V), Delta
#     = kappa/2 (0.92 Lx)^2 shrinks by it, and g shrinks by scale^2 (the shell's
#     area and so its norm-1 density change by scale^2; g |psi|^2, the Thomas-
#     Fermi thickness and the stable dt stay those of the full shell).
def c5_subdomain(scale: int = 8, box_n=(2048, 2048, 1024), h: float = 0.0306, seed: int = 5) -> Workload:
    n = tuple(int(v) // int(scale) for v in box_n)
    box = Box.centred(n, tuple(0.5 * v * h for v in n))
    kappa, omega, cut = 12.9 * scale, 2.0, 61.0
    Lx = 0.5 * n[0] * h
    delta = 0.5 * kappa * (0.92 * Lx) ** 2
    g = 1e4 / float(scale) ** 2
    lo, hi = rf_window(delta, omega, cut)
    runs = _rf_runs(box, kappa, lo, hi)
    U = _rf_U(box, runs, kappa)
    V = np.sqrt((U - delta) ** 2 + omega ** 2)
    rng = np.random.default_rng(seed)
    psi = tf_trial(V, omega + 20.0, g, box.dV, rng, 1e-3)
    return Workload(f"C5 subdomain {n[0]}x{n[1]}x{n[2]} h={h} (C5 / {scale})", box, runs, U, "rf",
                    omega=omega, knot_t=np.array([0.0]), knot_delta=np.array([delta]),
                    g=g, dt=5e-5, steps=20000, psi0=psi, extra={"scale": int(scale)})


# ----------------------------------------------------------------------------
# Small seeded problems for tests.
# ----------------------------------------------------------------------------
def random_mask_problem(n=(10, 9, 12), density: float = 0.6, seed: int = 7, g: float = 50.0,
                        h=(0.5, 0.45, 0.4)) -> Workload:
    """A ragged random mask (isolated sites, 1-site runs, runs on every face)."""
    rng = np.random.default_rng(seed)
    box = Box(tuple(n), tuple(h), tuple(-0.5 * n[d] * h[d] + 0.5 * h[d] for d in range(3)))
    mask = rng.random(n) < density
    runs = runs_from_mask(mask)
    V = rng.uniform(0.0, 5.0, size=int(mask.sum()))
    psi = complex_noise(rng, V.size, 1.0)
    psi = normalise_input(psi, box.dV)
    return Workload(f"random mask {n} p={density}", box, runs, V, "static", g=g, dt=1e-3, steps=10,
                    psi0=psi, extra={"mask": mask})


def full_box_problem(n=8, half_width=2.0, g: float = 10.0, seed: int = 11) -> Workload:
    box = Box.centred(n, half_width)
    mask = np.ones(box.n, bool)
    runs = runs_from_mask(mask)
    x, y, z = site_coords(box, runs)
    V = 0.5 * (x * x + y * y + z * z)
    rng = np.random.default_rng(seed)
    psi = np.exp(-(x * x + y * y + z * z) / 2.0) + complex_noise(rng, V.size, 1e-2)
    psi = normalise_input(psi, box.dV)
    return Workload(f"full box {n}^3", box, runs, V, "static", g=g, dt=1e-3, steps=10, psi0=psi,
                    extra={"mask": mask})


def small_shell(n: int = 24, half_width: float = 6.0, lam: float = 40.0, R0: float = 3.5,
                cut: float = 20.0, g: float = 100.0, seed: int = 0) -> Workload:
    """A C1-like shell on a smaller box (several tiles and ragged tails)."""
    box = Box.centred(n, half_width)

    def active(x, y, z):
        r = np.sqrt(x * x + y * y + z * z)
        return 0.5 * lam * (r - R0) ** 2 < cut

    runs = runs_from_predicate(box, active)
    x, y, z = site_coords(box, runs)
    r = np.sqrt(x * x + y * y + z * z)
    V = 0.5 * lam * (r - R0) ** 2
    rng = np.random.default_rng(seed)
    psi = np.exp(-np.sqrt(lam) * (r - R0) ** 2 / 2.0) + complex_noise(rng, r.size, 1e-3)
    psi = normalise_input(psi, box.dV)
    return Workload(f"shell {n}^3", box, runs, V, "static", g=g, dt=1e-3, steps=20, psi0=psi)


def small_rf_ramp(n: int = 32, half_width: float = 6.4, steps: int = 40, g: float = 300.0,
                  seed: int = 21, n_knots: int = 8) -> Workload:
    """A C3-like hollowing ramp on a small box (for RK4/adjoint parity)."""
    box = Box.centred(n, half_width)
    kappa = (12.8 / (2 * half_width)) ** 2 * 4.0
    omega, cut = 2.0, 20.0
    d0, d1 = -5.0, 15.0
    lo, _ = rf_window(d0, omega, cut)
    _, hi = rf_window(d1, omega, cut)
    runs = _rf_runs(box, kappa, lo, hi)
    U = _rf_U(box, runs, kappa)
    dt = 2e-3
    T = dt * steps
    rng = np.random.default_rng(seed)
    V0 = np.sqrt((U - d0) ** 2 + omega ** 2)
    psi = tf_trial(V0, np.min(V0) + 6.0, g, box.dV, rng, 1e-2)
    kd = np.linspace(d0, d1, n_knots) + rng.uniform(-1.0, 1.0, n_knots)
    return Workload(f"rf ramp {n}^3", box, runs, U, "rf", omega=omega,
                    knot_t=np.linspace(0.0, T, n_knots), knot_delta=kd, g=g, dt=dt, steps=steps, psi0=psi)


@dataclass
class StagedRamp:
    """Inputs of a staged ramp (Sec. V): stage potentials on the whole box,
    their chemical potentials, and a start state on the whole box."""
    name: str
    box: Box
    fields: list            # V_0 .. V_S, each a box array (n0, n1, n2)
    mus: list               # mu_0 .. mu_S
    g: float
    dt: float
    steps_per_stage: int
    psi0_box: np.ndarray    # complex box array


def staged_rf_shells(n: int = 24, half_width: float = 6.0, n_stages: int = 3, steps_per_stage: int = 12,
                     g: float = 60.0, seed: int = 7) -> StagedRamp:
    """A small hollowing ramp given as stage arrays: RF-dressed shells
    sqrt((U - Delta_i)^2 + Omega^2), U = (x^2 + y^2 + 4 z^2)/2, with Delta_i
    stepped from 2 to 9; stage chemical potentials grow slowly with i."""
    box = Box.centred(n, half_width)
    ax = [box.axis(d) for d in range(3)]
    x, y, z = np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
    U = 0.5 * (x * x + y * y + 4.0 * z * z)
    omega = 1.5
    deltas = np.linspace(2.0, 9.0, n_stages + 1)
    fields = [np.sqrt((U - d) ** 2 + omega ** 2) for d in deltas]
    mus = [2.5 + 0.2 * i for i in range(n_stages + 1)]
    rng = np.random.default_rng(seed)
    psi = tf_trial(fields[0].ravel(), mus[0], g, box.dV, rng, 1e-3).reshape(box.n)
    return StagedRamp(f"staged rf shells {n}^3", box, fields, mus, g, 2e-3, steps_per_stage, psi)
