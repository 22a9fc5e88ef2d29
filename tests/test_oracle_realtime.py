"""Pins for the oracle's real-time RK4 (Sec. II.A, eqs. (8)-(9); App. A)."""
import numpy as np
import pytest

from oracle import operator as op
from oracle import realtime as rt, observables as ob, dense, tableau
from oracle.potential import StaticPotential, RFRamp
from workloads import configs, site_linear_index


def _setup(w):
    lin = site_linear_index(w.box, w.runs)
    return lin, op.kinetic_direct(w.box.n, w.box.h, lin)


def test_linear_case_equals_rk4_stability_polynomial():
    """g = 0, static V: one RK4 step is R(-i H dt) with R(z) = 1 + z + z^2/2 +
    z^3/6 + z^4/24, so n steps are W R(-i lam dt)^n W^T psi0 (eigh of H~)."""
    w = configs.random_mask_problem(n=(6, 5, 7), density=0.6, seed=5)
    lin, T = _setup(w)
    H = T.toarray() + np.diag(w.field)
    lam, W = np.linalg.eigh(H)
    dt, n = 0.01, 60
    z = -1j * lam * dt
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    c = W.T @ w.psi0
    exact = W @ (R ** n * c)
    got = rt.real_time(T, w.psi0, StaticPotential(w.field), 0.0, dt, 0.0, n)
    assert np.linalg.norm(got - exact) <= 1e-12 * np.linalg.norm(exact)
    # norm after n steps: sum_k |c_k|^2 |R_k|^(2n) dV
    assert abs(ob.norm(got, w.box.dV) - np.sum(np.abs(c) ** 2 * np.abs(R) ** (2 * n)) * w.box.dV) < 1e-13


def _ramp_problem():
    w = configs.small_rf_ramp(n=16, half_width=6.4, steps=20, g=200.0)
    lin, T = _setup(w)
    ramp = RFRamp(w.field, w.omega, w.knot_t, w.knot_delta)
    return w, T, ramp


def test_fourth_order_convergence_with_time_dependent_potential():
    """Halving dt divides the global error by ~16 (order 4).  Using the wrong
    stage times c_i would drop the order, so this also pins c = (0, 1/2, 1/2, 1)."""
    w, T, ramp = _ramp_problem()
    Tend = 0.04
    # a single linear ramp segment: V(t) is smooth in t (kinks of a
    # piecewise-linear ramp inside a step would lower the observed order)
    ramp = RFRamp(w.field, w.omega, [0.0, Tend], [-5.0, 15.0])
    ref = rt.real_time(T, w.psi0, ramp, w.g, Tend / 512, 0.0, 512)
    errs = []
    for m in (16, 32, 64):
        y = rt.real_time(T, w.psi0, ramp, w.g, Tend / m, 0.0, m)
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13.0 < r1 < 19.0 and 13.0 < r2 < 19.0, (errs, r1, r2)


def test_norm_and_energy_conservation_static():
    w = configs.small_shell(n=16, half_width=6.0, R0=3.5, g=100.0)
    lin, T = _setup(w)
    pot = StaticPotential(w.field)
    N0, E0, _ = ob.energy_mu(T, w.psi0, w.field, w.g, w.box.dV)
    drifts = []
    for dt in (2e-3, 1e-3):
        y = rt.real_time(T, w.psi0, pot, w.g, dt, 0.0, int(round(0.1 / dt)))
        N1, E1, _ = ob.energy_mu(T, y, w.field, w.g, w.box.dV)
        drifts.append((abs(N1 - N0), abs(E1 - E0) / abs(E0)))
    assert drifts[1][0] < 1e-8 and drifts[1][1] < 1e-7
    assert drifts[0][0] / drifts[1][0] > 10.0      # >= 4th-order-ish decay of the drift


def test_masked_equals_dense_projector():
    w = configs.random_mask_problem(n=(6, 5, 6), density=0.6, seed=12, g=20.0)
    mask = w.extra["mask"]
    lin, T = _setup(w)
    y = rt.real_time(T, w.psi0, StaticPotential(w.field), w.g, 0.004, 0.0, 25)
    Vbox = np.zeros(w.box.n)
    Vbox.ravel()[lin] = w.field
    p0 = np.zeros(w.box.n, complex)
    p0.ravel()[lin] = w.psi0
    ref = dense.dense_rk4(w.box.n, w.box.h, mask, lambda t: Vbox, p0, w.g, 0.004, 0.0, 25).ravel()
    assert np.max(np.abs(ref[~mask.ravel()])) == 0.0
    assert np.linalg.norm(y - ref[lin]) <= 1e-13 * np.linalg.norm(ref)


def test_memory_optimised_form_equals_classic():
    """App. A: y^(i+1) = sum_j a*_ij y^(j) + dt a_{i+1,i} k_i and
    y_1 = sum_j b*_j y^(j) + dt b_n k_n, with (a*, b*) derived exactly from
    the classic tableau, reproduce the classic RK4 step to rounding."""
    w, T, ramp = _ramp_problem()
    A, b = tableau.rk4()
    a_star, b_star = tableau.modified_tableau(A, b)
    c = [0.0, 0.5, 0.5, 1.0]
    y0, t, dt = w.psi0, 0.013, 2e-3
    Y = [y0]
    for i in range(4):
        k = rt.rhs(T, ramp(t + c[i] * dt), w.g, Y[i])
        if i < 3:
            nxt = sum(float(a_star[i][j]) * Y[j] for j in range(i + 1)) + dt * float(A[i + 1][i]) * k
            Y.append(nxt)
        else:
            y1 = sum(float(b_star[j]) * Y[j] for j in range(4)) + dt * float(b[3]) * k
    ref = rt.rk4_step(T, y0, t, dt, ramp, w.g)
    assert np.linalg.norm(y1 - ref) <= 1e-14 * np.linalg.norm(ref)


METHODS = [("RKHE3", tableau.heun3, 3), ("RK4", tableau.rk4, 4), ("RKCK", tableau.cash_karp5, 5)]


@pytest.mark.parametrize("name,fn,order", METHODS)
def test_tableau_method_linear_case_equals_stability_function(name, fn, order):
    """g = 0, static V: one step of an explicit method is y -> R(-i H dt) y with
    the stability function R(z) = 1 + z b^T (I - z A)^-1 e."""
    A, b = fn()
    Af = np.array([[float(v) for v in r] for r in A])
    bf = np.array([float(v) for v in b])
    w = configs.random_mask_problem(n=(5, 6, 5), density=0.6, seed=15)
    lin, T = _setup(w)
    H = T.toarray() + np.diag(w.field)
    lam, W = np.linalg.eigh(H)
    dt, n = 0.01, 40
    e = np.ones(len(bf))
    R = np.array([1 + z * bf @ np.linalg.solve(np.eye(len(bf)) - z * Af, e) for z in -1j * lam * dt])
    exact = W @ (R ** n * (W.T @ w.psi0))
    got = rt.real_time_tableau(T, w.psi0, StaticPotential(w.field), 0.0, dt, 0.0, n, A, b)
    assert np.linalg.norm(got - exact) <= 1e-12 * np.linalg.norm(exact)
    # R agrees with exp(z) to the method's order
    z = 1e-2j
    Rz = 1 + z * bf @ np.linalg.solve(np.eye(len(bf)) - z * Af, e)
    assert abs(Rz - np.exp(z)) < 10 * abs(z) ** (order + 1)


@pytest.mark.parametrize("name,fn,order", METHODS)
def test_tableau_method_convergence_order(name, fn, order):
    w, T, ramp = _ramp_problem()
    A, b = fn()
    Tend = 0.04
    ramp = RFRamp(w.field, w.omega, [0.0, Tend], [-5.0, 15.0])
    ref = rt.real_time_tableau(T, w.psi0, ramp, w.g, Tend / 256, 0.0, 256, *tableau.cash_karp5())
    errs = []
    for m in (8, 16, 32):
        y = rt.real_time_tableau(T, w.psi0, ramp, w.g, Tend / m, 0.0, m, A, b)
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    r = errs[1] / errs[2]
    assert 0.75 * 2 ** order < r < 1.3 * 2 ** order, (errs, r)


def test_rk4_tableau_equals_rk4_step():
    w, T, ramp = _ramp_problem()
    a = rt.rk4_step(T, w.psi0, 0.01, 2e-3, ramp, w.g)
    b_ = rt.rk_step_tableau(T, w.psi0, 0.01, 2e-3, ramp, w.g, *tableau.rk4())
    assert np.linalg.norm(a - b_) <= 1e-15 * np.linalg.norm(a)


@pytest.mark.parametrize("name,fn,order", METHODS)
def test_memory_optimised_form_of_each_method(name, fn, order):
    """App. A form with the derived (a*, b*) reproduces the k-form step."""
    w, T, ramp = _ramp_problem()
    A, b = fn()
    a_star, b_star = tableau.modified_tableau(A, b)
    c = [float(sum(r)) for r in A]
    y0, t, dt = w.psi0, 0.013, 2e-3
    Y = [y0]
    s = len(b)
    for i in range(s):
        k = rt.rhs(T, ramp(t + c[i] * dt), w.g, Y[i])
        if i < s - 1:
            Y.append(sum(float(a_star[i][j]) * Y[j] for j in range(i + 1)) + dt * float(A[i + 1][i]) * k)
        else:
            y1 = sum(float(b_star[j]) * Y[j] for j in range(s)) + dt * float(b[s - 1]) * k
    ref = rt.rk_step_tableau(T, y0, t, dt, ramp, w.g, A, b)
    assert np.linalg.norm(y1 - ref) <= 1e-13 * np.linalg.norm(ref)


def test_ground_state_only_turns_its_phase_at_mu():
    """A converged ground state psi_0 (H psi_0 = mu psi_0 with H = T + V +
    g|psi_0|^2) evolves in real time as exp(-i mu t) psi_0: the density
    stays put and the overlap with psi_0 turns at the rate mu.  The ground
    state is the imaginary-time fixed point at a small step, which solves the
    eigen-equation up to O(dt_itp); a nonlinearity of weight 2g in the
    right-hand side misses the phase by 30 %."""
    from oracle import itp
    from workloads import Box, runs_from_mask, site_coords, normalise_input
    box = Box.centred(16, 4.0)
    runs = runs_from_mask(np.ones(box.n, bool))
    lin = site_linear_index(box, runs)
    T = op.kinetic_direct(box.n, box.h, lin)
    x, y, z = site_coords(box, runs)
    V = 0.5 * (x * x + y * y + z * z)
    g = 20.0
    psi0 = normalise_input(np.exp(-0.5 * (x * x + y * y + z * z)).astype(complex), box.dV)
    gs, _ = itp.imaginary_time(T, psi0, V, g, 1e-3, box.dV, 8000)
    _, E, mu = ob.energy_mu(T, gs, V, g, box.dV)
    t = 0.2
    yt = rt.real_time(T, gs, StaticPotential(V), g, 1e-3, 0.0, 200)
    d0 = np.abs(gs) ** 2
    assert np.linalg.norm(np.abs(yt) ** 2 - d0) / np.linalg.norm(d0) <= 5e-4      # measured 5.0e-5
    ov = np.vdot(gs, yt) / np.vdot(gs, gs)
    assert abs(abs(ov) - 1.0) <= 1e-6                                               # measured 3.9e-9
    assert abs(np.angle(ov) + mu * t) <= 1e-4 * mu * t, (np.angle(ov), -mu * t)      # measured 2.2e-6
