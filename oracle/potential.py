"""Potentials (oracle; test infrastructure).

Eq. (10): an RF-dressed adiabatic potential V = hbar m_F sqrt(delta^2 + Omega^2),
where delta is the detuning from the local Larmor frequency.  In the
dimensionless form used here the bare trap U(x) plays the role of the local
Larmor frequency and Delta is the RF detuning at the trap centre, so
V(x, t) = sqrt((U(x) - Delta(t))^2 + Omega^2).

Sec. V ramps the detuning through a sequence of stages with the potential
interpolated linearly in time between them; here Delta(t) is the
piecewise-linear interpolant of knot values Delta_k at times t_k, held
constant before the first and after the last knot.  The same kind of ramp
drives the radius R0(t) of a harmonic shell lambda/2 (r - R0)^2 (ShellRamp).
"""
from __future__ import annotations

import numpy as np


def delta_at(t: float, knot_t, knot_delta) -> float:
    return float(np.interp(t, np.asarray(knot_t, float), np.asarray(knot_delta, float)))


def hat_weights(t: float, knot_t) -> np.ndarray:
    """d Delta(t) / d Delta_k for every knot k (the piecewise-linear hat functions)."""
    kt = np.asarray(knot_t, float)
    e = np.eye(kt.size)
    return np.array([np.interp(t, kt, e[k]) for k in range(kt.size)])


def rf_potential(U: np.ndarray, delta: float, omega: float) -> np.ndarray:
    return np.sqrt((U - delta) ** 2 + omega * omega)


def rf_dV_ddelta(U: np.ndarray, delta: float, omega: float) -> np.ndarray:
    """Derivative of eq. (10) with respect to the detuning Delta."""
    return -(U - delta) / np.sqrt((U - delta) ** 2 + omega * omega)


def shell_potential(r: np.ndarray, radius: float, lam: float) -> np.ndarray:
    """Harmonic shell V = lambda/2 (r - R0)^2 (the shell of the C1 workload)."""
    return 0.5 * lam * (r - radius) ** 2


def shell_dV_dradius(r: np.ndarray, radius: float, lam: float) -> np.ndarray:
    """Derivative of the harmonic shell with respect to its radius R0."""
    return -lam * (r - radius)


class StaticPotential:
    def __init__(self, V: np.ndarray):
        self.V = np.asarray(V, float)

    def __call__(self, t: float) -> np.ndarray:
        return self.V


class RFRamp:
    def __init__(self, U: np.ndarray, omega: float, knot_t, knot_delta):
        self.U = np.asarray(U, float)
        self.omega = float(omega)
        self.knot_t = np.asarray(knot_t, float)
        self.knot_delta = np.asarray(knot_delta, float)

    def delta(self, t: float) -> float:
        return delta_at(t, self.knot_t, self.knot_delta)

    def __call__(self, t: float) -> np.ndarray:
        return rf_potential(self.U, self.delta(t), self.omega)

    def dV_ddelta(self, t: float) -> np.ndarray:
        return rf_dV_ddelta(self.U, self.delta(t), self.omega)

    def with_knots(self, knot_delta) -> "RFRamp":
        return RFRamp(self.U, self.omega, self.knot_t, knot_delta)


class ShellRamp:
    """Harmonic shell V(x, t) = lambda/2 (r(x) - R0(t))^2 whose radius R0(t) is
    the piecewise-linear interpolant of knot values (held before the first
    and after the last knot): a shell inflated over the run, ramped like
    Delta(t) of eq. (10) in Sec. V.  `r` is the distance of each site from
    the shell's centre."""

    def __init__(self, r: np.ndarray, lam: float, knot_t, knot_radius):
        self.r = np.asarray(r, float)
        self.lam = float(lam)
        self.knot_t = np.asarray(knot_t, float)
        self.knot_delta = np.asarray(knot_radius, float)

    def delta(self, t: float) -> float:
        return delta_at(t, self.knot_t, self.knot_delta)

    def __call__(self, t: float) -> np.ndarray:
        return shell_potential(self.r, self.delta(t), self.lam)

    def dV_ddelta(self, t: float) -> np.ndarray:
        return shell_dV_dradius(self.r, self.delta(t), self.lam)

    def with_knots(self, knot_radius) -> "ShellRamp":
        return ShellRamp(self.r, self.lam, self.knot_t, knot_radius)
