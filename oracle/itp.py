"""Imaginary-time propagation with renormalisation (oracle; test infrastructure).

Sec. II.A, eqs. (6)-(7) and the footnote on the kinetic step.  One step of
length dt, for the reduced vectors psi~, V~ and operator T~:

1. diagonal half-step, eq. (7): psi <- psi * exp(-V dt/2) * (1 - g|psi|^2 dt/2)
   (the interaction exponential replaced by its linearisation, as the paper
   does for dilute condensates; |psi|^2 is taken from the half-step's input
   and used in that one factor);
2. kinetic propagation for a total time dt in two forward-Euler substeps:
   chi = phi - (dt/2) T~ phi,  chi' = chi - (dt/2) T~ chi;
3. a second diagonal half-step as in 1;
4. renormalise so that dV * sum |psi|^2 = N (eq. (3)).

The paper writes the half-step for a real psi (psi^2); for complex psi the
modulus |psi|^2 is used.  exp(-V dt/2) is precomputed once, as the paper
recommends.
"""
from __future__ import annotations

import numpy as np

from .operator import apply
from .observables import energy_mu


def propagator(V: np.ndarray, dt: float) -> np.ndarray:
    return np.exp(-V * dt / 2.0)


def diagonal_half_step(psi: np.ndarray, P: np.ndarray, g: float, dt: float) -> np.ndarray:
    dens = psi.real ** 2 + psi.imag ** 2
    return psi * P * (1.0 - g * dens * dt / 2.0)


def itp_step(T, psi, P, g, dt, dV, norm_target=1.0):
    phi = diagonal_half_step(psi, P, g, dt)
    chi = phi - (dt / 2.0) * apply(T, phi)
    chi = chi - (dt / 2.0) * apply(T, chi)
    omega = diagonal_half_step(chi, P, g, dt)
    n = float(np.sum(omega.real ** 2 + omega.imag ** 2)) * dV
    return omega * np.sqrt(norm_target / n), n


def imaginary_time(T, psi0, V, g, dt, dV, steps, norm_target=1.0, observe_every=0):
    """Run `steps` steps.  Returns (psi, history) with history a list of
    (step, N, E, mu) rows evaluated every `observe_every` steps (before the
    step), if requested."""
    P = propagator(np.asarray(V, float), dt)
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    hist = []
    for s in range(steps):
        if observe_every and s % observe_every == 0:
            hist.append((s,) + energy_mu(T, psi, V, g, dV))
        psi, _ = itp_step(T, psi, P, g, dt, dV, norm_target)
    return psi, hist
