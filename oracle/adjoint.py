"""Discrete adjoint of the RK4 map for a ramp-fidelity loss (oracle; test
infrastructure).

The paper optimises ramp timings without gradients (Sec. V, Bayesian
optimisation); it is silent on adjoints.  What is computed here is the exact
gradient of the *discrete* forward map of realtime.rk4_step with respect to
the knot values Delta_k of the detuning ramp (Sec. V; potential eq. (10)).

Loss: L = 1 - |c|^2 with c = <psi_target | psi(T)> = dV sum conj(psi_T) psi_N.

Real inner product on complex vectors: <a, b>_R = Re sum conj(a) b.  The
gradient lambda of a real function F of complex y is defined by
dF = <lambda, dy>_R.  Seed: dL = -2 Re(conj(c) dc) gives
lambda_N = -2 dV c psi_T.

Right-hand side f(t, y) = -i [H(t) y + g |y|^2 y] with H = T~ + V(t) real
symmetric.  Its real-linear Jacobian at Y is
    J d = -i [ (H + 2 g |Y|^2) d + g Y^2 conj(d) ],
and the transpose with respect to <.,.>_R is
    J^T u = i (H + 2 g |Y|^2) u - i g Y^2 conj(u).

One RK4 step y' = y + dt sum_i b_i k_i, k_i = f(t + c_i dt, Y_i),
Y_i = y + dt sum_{j<i} a_ij k_j (a_21 = a_32 = 1/2, a_43 = 1) is reversed as
    u_4 = b_4 lam,                 theta_4 = dt J_4^T u_4
    u_i = b_i lam + a_{i+1,i} theta_{i+1},   theta_i = dt J_i^T u_i   (i = 3, 2, 1)
    lam <- lam + theta_1 + theta_2 + theta_3 + theta_4
and the parameter gradient of the step is
    dL/dDelta_k += dt sum_i phi_k(t + c_i dt) < -i (dV/dDelta)(t_i) Y_i , u_i >_R,
where phi_k is the hat function of knot k (d Delta(t)/d Delta_k).

Forward states are stored every K = ceil(sqrt(N)) steps; during the reverse
sweep each segment of K steps is recomputed from its checkpoint.
"""
from __future__ import annotations

import math

import numpy as np

from .operator import apply
from .potential import hat_weights
from .realtime import rhs, rk4_step

RK4_A_SUB = (0.5, 0.5, 1.0)          # a_21, a_32, a_43
RK4_B = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)
RK4_C = (0.0, 0.5, 0.5, 1.0)


def jacobian(T, V, g, Y, d):
    return -1j * (apply(T, d) + (V + 2.0 * g * np.abs(Y) ** 2) * d + g * Y * Y * np.conj(d))


def jacobian_T(T, V, g, Y, u):
    return 1j * (apply(T, u) + (V + 2.0 * g * np.abs(Y) ** 2) * u) - 1j * g * Y * Y * np.conj(u)


def real_inner(a, b) -> float:
    return float(np.sum(a.real * b.real + a.imag * b.imag))


def stages(T, y, t, dt, ramp, g):
    Ys = [y]
    ks = []
    for i in range(4):
        ti = t + RK4_C[i] * dt
        ks.append(rhs(T, ramp(ti), g, Ys[i]))
        if i < 3:
            Ys.append(y + dt * RK4_A_SUB[i] * ks[i])
    return Ys


def adjoint_step(T, y, t, dt, ramp, g, lam):
    """Reverse one RK4 step that started from y at time t.  Returns the new
    lambda and the step's contribution to dL/dDelta_k."""
    Ys = stages(T, y, t, dt, ramp, g)
    nk = ramp.knot_t.size
    grad = np.zeros(nk)
    theta_next = None
    lam_new = lam.copy()
    for i in (3, 2, 1, 0):
        u = RK4_B[i] * lam
        if theta_next is not None:
            u = u + RK4_A_SUB[i] * theta_next
        ti = t + RK4_C[i] * dt
        theta = dt * jacobian_T(T, ramp(ti), g, Ys[i], u)
        q = real_inner(-1j * ramp.dV_ddelta(ti) * Ys[i], u)
        grad += dt * hat_weights(ti, ramp.knot_t) * q
        lam_new = lam_new + theta
        theta_next = theta
    return lam_new, grad


def fidelity_loss(T, ramp, g, dt, t0, steps, psi0, psi_target, dV):
    y = np.array(psi0, dtype=np.complex128, copy=True)
    for n in range(steps):
        y = rk4_step(T, y, t0 + n * dt, dt, ramp, g)
    c = complex(np.sum(np.conj(psi_target) * y)) * dV
    return 1.0 - abs(c) ** 2, y


def fidelity_grad(T, ramp, g, dt, t0, steps, psi0, psi_target, dV, ckpt_every=0):
    """Loss, gradient with respect to the knot values, and the final state."""
    K = int(ckpt_every) if ckpt_every else max(1, math.ceil(math.sqrt(steps)))
    ckpts = {}
    y = np.array(psi0, dtype=np.complex128, copy=True)
    for n in range(steps):
        if n % K == 0:
            ckpts[n] = y.copy()
        y = rk4_step(T, y, t0 + n * dt, dt, ramp, g)
    c = complex(np.sum(np.conj(psi_target) * y)) * dV
    loss = 1.0 - abs(c) ** 2
    lam = -2.0 * dV * c * np.asarray(psi_target, np.complex128)
    grad = np.zeros(ramp.knot_t.size)
    nseg = (steps + K - 1) // K
    for m in reversed(range(nseg)):
        n0, n1 = m * K, min(m * K + K, steps)
        seg = [ckpts[n0]]
        for n in range(n0, n1 - 1):
            seg.append(rk4_step(T, seg[-1], t0 + n * dt, dt, ramp, g))
        for n in reversed(range(n0, n1)):
            lam, gs = adjoint_step(T, seg[n - n0], t0 + n * dt, dt, ramp, g, lam)
            grad += gs
    return loss, grad, y
