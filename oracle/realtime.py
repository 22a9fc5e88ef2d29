"""Real-time evolution with explicit Runge-Kutta methods (oracle; test
infrastructure).

Sec. II.A, eq. (8): d psi~/dt = -i (T~ + V~(t) + g |psi~|^2) psi~ (hbar = 1),
integrated with an explicit Runge-Kutta method without splitting.  Eq. (9):
k_i = f(t + c_i dt, y^(i)) with y^(i) = y_0 + dt sum_{j<i} a_ij k_j.

rk4_step is the standard k-form of RK4 (c = 0, 1/2, 1/2, 1; b = 1/6, 1/3,
1/3, 1/6); rk_step_tableau is the same k-form for any explicit tableau (the
paper also uses Heun's third-order method and the fifth-order Cash-Karp
weights).  Both are deliberately not the memory-optimised form of App. A.
"""
from __future__ import annotations

import numpy as np

from .operator import apply


def rhs(T, V, g, y):
    dens = y.real ** 2 + y.imag ** 2
    return -1j * (apply(T, y) + (V + g * dens) * y)


def rk4_step(T, y, t, dt, potential, g):
    k1 = rhs(T, potential(t), g, y)
    k2 = rhs(T, potential(t + dt / 2.0), g, y + (dt / 2.0) * k1)
    k3 = rhs(T, potential(t + dt / 2.0), g, y + (dt / 2.0) * k2)
    k4 = rhs(T, potential(t + dt), g, y + dt * k3)
    return y + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def rk_step_tableau(T, y, t, dt, potential, g, A, b):
    """One step of the explicit method with Butcher matrix A (strictly lower
    triangular) and weights b; stage times c_i = sum_j a_ij."""
    A = [[float(v) for v in row] for row in A]
    b = [float(v) for v in b]
    ks = []
    for i in range(len(b)):
        yi = y
        for j in range(i):
            if A[i][j] != 0.0:
                yi = yi + (dt * A[i][j]) * ks[j]
        ks.append(rhs(T, potential(t + sum(A[i]) * dt), g, yi))
    out = y
    for i in range(len(b)):
        if b[i] != 0.0:
            out = out + (dt * b[i]) * ks[i]
    return out


def real_time_tableau(T, psi0, potential, g, dt, t0, steps, A, b):
    y = np.array(psi0, dtype=np.complex128, copy=True)
    for n in range(steps):
        y = rk_step_tableau(T, y, t0 + n * dt, dt, potential, g, A, b)
    return y


def real_time(T, psi0, potential, g, dt, t0, steps, observe=None, observe_every=0):
    """Run `steps` RK4 steps from time t0.  `potential(t)` returns V~ at time t.
    Step n starts at t0 + n*dt.  If `observe` is given it is called as
    observe(n, t, y) every `observe_every` steps (before the step)."""
    y = np.array(psi0, dtype=np.complex128, copy=True)
    for n in range(steps):
        t = t0 + n * dt
        if observe is not None and observe_every and n % observe_every == 0:
            observe(n, t, y)
        y = rk4_step(T, y, t, dt, potential, g)
    return y
