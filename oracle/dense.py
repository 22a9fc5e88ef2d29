"""Dense Cartesian brute force on tiny boxes (oracle; test infrastructure).

The whole box is kept (no compaction).  The kinetic matrix is filled by
explicit loops over every grid point and its six neighbours, and the region
of interest enters only as a projector Pi (diagonal 0/1): T_Pi = Pi T Pi,
which is the same as dropping rows and columns outside the ROI (Sec. II.A)
while keeping zeros at the dropped points.  The imaginary-time and RK4
algebra is then applied with dense matrix products on full-box vectors.
Intended for boxes of at most ~12^3 points.
"""
from __future__ import annotations

import numpy as np


def dense_kinetic(n, h) -> np.ndarray:
    n0, n1, n2 = (int(v) for v in n)
    N = n0 * n1 * n2
    T = np.zeros((N, N))
    inv = [1.0 / (h[d] * h[d]) for d in range(3)]
    for i in range(n0):
        for j in range(n1):
            for k in range(n2):
                p = (i * n1 + j) * n2 + k
                T[p, p] = -0.5 * (-2.0) * (inv[0] + inv[1] + inv[2])
                for (di, dj, dk, w) in ((1, 0, 0, inv[0]), (-1, 0, 0, inv[0]),
                                        (0, 1, 0, inv[1]), (0, -1, 0, inv[1]),
                                        (0, 0, 1, inv[2]), (0, 0, -1, inv[2])):
                    a, b, c = i + di, j + dj, k + dk
                    if 0 <= a < n0 and 0 <= b < n1 and 0 <= c < n2:
                        T[p, (a * n1 + b) * n2 + c] = -0.5 * w
    return T


def projector(mask: np.ndarray) -> np.ndarray:
    return np.diag(np.asarray(mask, float).ravel())


def dense_itp(n, h, mask, Vbox, psi_box, g, dt, steps, norm_target=1.0):
    dV = h[0] * h[1] * h[2]
    Pi = projector(mask)
    TP = Pi @ dense_kinetic(n, h) @ Pi
    P = np.exp(-np.asarray(Vbox, float).ravel() * dt / 2.0) * np.asarray(mask, float).ravel()
    psi = np.asarray(psi_box, np.complex128).ravel() * np.asarray(mask, float).ravel()
    for _ in range(steps):
        d = np.abs(psi) ** 2
        phi = psi * P * (1.0 - g * d * dt / 2.0)
        chi = phi - (dt / 2.0) * (TP @ phi)
        chi = chi - (dt / 2.0) * (TP @ chi)
        d = np.abs(chi) ** 2
        om = chi * P * (1.0 - g * d * dt / 2.0)
        psi = om * np.sqrt(norm_target / (np.sum(np.abs(om) ** 2) * dV))
    return psi.reshape(n)


def dense_rk4(n, h, mask, Vbox_of_t, psi_box, g, dt, t0, steps):
    Pi = projector(mask)
    TP = Pi @ dense_kinetic(n, h) @ Pi
    m = np.asarray(mask, float).ravel()

    def f(t, y):
        V = np.asarray(Vbox_of_t(t), float).ravel() * m
        return -1j * (TP @ y + (V + g * np.abs(y) ** 2) * y)

    y = np.asarray(psi_box, np.complex128).ravel() * m
    for s in range(steps):
        t = t0 + s * dt
        k1 = f(t, y)
        k2 = f(t + dt / 2, y + dt / 2 * k1)
        k3 = f(t + dt / 2, y + dt / 2 * k2)
        k4 = f(t + dt, y + dt * k3)
        y = y + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y.reshape(n)
