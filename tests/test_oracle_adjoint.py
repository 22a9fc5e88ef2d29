"""Pins for the oracle's discrete adjoint (fidelity gradient w.r.t. ramp knots)."""
import numpy as np

from oracle import operator as op
from oracle import adjoint as adj, realtime as rt
from oracle.potential import RFRamp, ShellRamp, hat_weights
from workloads import configs, site_linear_index


def _problem(steps=12, n=14):
    w = configs.small_rf_ramp(n=n, half_width=6.4, steps=steps, g=250.0, n_knots=5)
    lin = site_linear_index(w.box, w.runs)
    T = op.kinetic_direct(w.box.n, w.box.h, lin)
    ramp = RFRamp(w.field, w.omega, w.knot_t, w.knot_delta)
    rng = np.random.default_rng(77)
    tgt = w.psi0 * np.exp(1j * rng.uniform(0, 0.3, w.psi0.size)) + 0.05 * rng.standard_normal(w.psi0.size)
    tgt = tgt / np.sqrt(np.sum(np.abs(tgt) ** 2) * w.box.dV)
    return w, T, ramp, tgt


def test_jacobian_matches_finite_differences_of_rhs():
    w, T, ramp, _ = _problem()
    rng = np.random.default_rng(3)
    y = w.psi0 * 3.0
    d = rng.standard_normal(y.size) + 1j * rng.standard_normal(y.size)
    V = ramp(0.01)
    eps = 1e-6
    fd = (rt.rhs(T, V, w.g, y + eps * d) - rt.rhs(T, V, w.g, y - eps * d)) / (2 * eps)
    J = adj.jacobian(T, V, w.g, y, d)
    assert np.linalg.norm(fd - J) <= 1e-8 * np.linalg.norm(J)


def test_transpose_dot_product():
    w, T, ramp, _ = _problem()
    rng = np.random.default_rng(4)
    Y = w.psi0 * 2.0
    v = rng.standard_normal(Y.size) + 1j * rng.standard_normal(Y.size)
    u = rng.standard_normal(Y.size) + 1j * rng.standard_normal(Y.size)
    V = ramp(0.0)
    lhs = adj.real_inner(adj.jacobian(T, V, w.g, Y, v), u)
    rhs_ = adj.real_inner(v, adj.jacobian_T(T, V, w.g, Y, u))
    assert abs(lhs - rhs_) <= 1e-12 * abs(lhs)


def test_hat_weights_sum_and_interpolate():
    kt = np.array([0.0, 0.1, 0.25, 0.4])
    kd = np.array([1.0, -2.0, 5.0, 3.0])
    for t in (-0.1, 0.0, 0.05, 0.1, 0.2, 0.4, 0.7):
        wts = hat_weights(t, kt)
        assert abs(wts.sum() - 1.0) < 1e-15
        assert abs(wts @ kd - np.interp(t, kt, kd)) < 1e-14


def test_gradient_matches_central_differences():
    w, T, ramp, tgt = _problem()
    loss, grad, _ = adj.fidelity_grad(T, ramp, w.g, w.dt, 0.0, w.steps, w.psi0, tgt, w.box.dV)
    assert 0.0 < loss < 1.0
    h = 1e-5
    for k in range(ramp.knot_t.size):
        kp = ramp.knot_delta.copy(); kp[k] += h
        km = ramp.knot_delta.copy(); km[k] -= h
        lp, _ = adj.fidelity_loss(T, ramp.with_knots(kp), w.g, w.dt, 0.0, w.steps, w.psi0, tgt, w.box.dV)
        lm, _ = adj.fidelity_loss(T, ramp.with_knots(km), w.g, w.dt, 0.0, w.steps, w.psi0, tgt, w.box.dV)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-6 * np.max(np.abs(grad)) + 1e-11, (k, fd, grad[k])


def test_checkpoint_interval_does_not_change_result():
    w, T, ramp, tgt = _problem(steps=10)
    outs = [adj.fidelity_grad(T, ramp, w.g, w.dt, 0.0, w.steps, w.psi0, tgt, w.box.dV, ckpt_every=K)
            for K in (1, 3, 0, 10)]
    for loss, grad, y in outs[1:]:
        assert loss == outs[0][0]
        assert np.array_equal(grad, outs[0][1])
        assert np.array_equal(y, outs[0][2])


def _shell_problem(steps=10, n=12):
    w = configs.c4_instance(3, n_lo=n, n_hi=n, steps=steps)
    w.g = 40.0
    lin = site_linear_index(w.box, w.runs)
    T = op.kinetic_direct(w.box.n, w.box.h, lin)
    ramp = ShellRamp(w.field, w.omega, w.knot_t, w.knot_delta)
    rng = np.random.default_rng(78)
    tgt = w.psi0 * np.exp(1j * rng.uniform(0, 0.3, w.psi0.size)) + 0.05 * rng.standard_normal(w.psi0.size)
    tgt = tgt / np.sqrt(np.sum(np.abs(tgt) ** 2) * w.box.dV)
    return w, T, ramp, tgt


def test_shell_ramp_potential_and_radius_derivative():
    """V = lambda/2 (r - R0(t))^2 with R0(t) the knot interpolant, and dV/dR0
    equal to a central difference of V in the radius."""
    w, _, ramp, _ = _shell_problem()
    t = 0.37 * w.knot_t[-1]
    R0 = np.interp(t, w.knot_t, w.knot_delta)
    assert np.allclose(ramp(t), 0.5 * w.omega * (w.field - R0) ** 2, rtol=1e-15, atol=0)
    eps = 1e-6
    up = ShellRamp(w.field, w.omega, w.knot_t, w.knot_delta + eps)(t)
    dn = ShellRamp(w.field, w.omega, w.knot_t, w.knot_delta - eps)(t)
    assert np.max(np.abs((up - dn) / (2 * eps) - ramp.dV_ddelta(t))) <= 1e-6 * np.max(np.abs(ramp.dV_ddelta(t)))


def test_shell_ramp_gradient_matches_central_differences():
    """The same discrete adjoint with the radius of a harmonic shell as the
    ramped parameter."""
    w, T, ramp, tgt = _shell_problem()
    loss, grad, _ = adj.fidelity_grad(T, ramp, w.g, w.dt, 0.0, w.steps, w.psi0, tgt, w.box.dV)
    assert 0.0 < loss < 1.0
    h = 1e-5
    fd = np.zeros(ramp.knot_t.size)
    for k in range(ramp.knot_t.size):
        kp = ramp.knot_delta.copy(); kp[k] += h
        km = ramp.knot_delta.copy(); km[k] -= h
        lp, _ = adj.fidelity_loss(T, ramp.with_knots(kp), w.g, w.dt, 0.0, w.steps, w.psi0, tgt, w.box.dV)
        lm, _ = adj.fidelity_loss(T, ramp.with_knots(km), w.g, w.dt, 0.0, w.steps, w.psi0, tgt, w.box.dV)
        fd[k] = (lp - lm) / (2 * h)
    assert np.max(np.abs(fd - grad)) <= 1e-6 * np.max(np.abs(grad))
