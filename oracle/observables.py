"""Particle number, energy and chemical potential (oracle; test infrastructure).

Eq. (3): N = integral |psi|^2 dV, here dV * sum |psi|^2 over the active set.
Energy functional of eqs. (1)-(2) on the reduced grid:
    E  = dV [ Re psi^H T~ psi + sum V |psi|^2 + g/2 sum |psi|^4 ] / N
    mu = dV [ Re psi^H T~ psi + sum V |psi|^2 + g   sum |psi|^4 ] / N
(mu is the Rayleigh quotient of the left-hand side of eq. (1)).
"""
from __future__ import annotations

import numpy as np

from .operator import apply


def norm(psi: np.ndarray, dV: float) -> float:
    return float(np.sum(psi.real ** 2 + psi.imag ** 2)) * dV


def energy_mu(T, psi: np.ndarray, V: np.ndarray, g: float, dV: float):
    dens = psi.real ** 2 + psi.imag ** 2
    N = float(np.sum(dens)) * dV
    Tpsi = apply(T, psi)
    kin = float(np.sum(psi.real * Tpsi.real + psi.imag * Tpsi.imag))
    pot = float(np.sum(V * dens))
    inter = float(np.sum(dens * dens))
    E = dV * (kin + pot + 0.5 * g * inter) / N
    mu = dV * (kin + pot + g * inter) / N
    return N, E, mu


def overlap(a: np.ndarray, b: np.ndarray, dV: float) -> complex:
    """<a|b> = dV sum conj(a) b."""
    return complex(np.sum(np.conj(a) * b)) * dV
