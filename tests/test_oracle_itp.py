"""Pins for the oracle's imaginary-time propagation (Sec. II.A, eqs. (6)-(7))."""
import numpy as np
import pytest

from oracle import operator as op
from oracle import itp, observables as ob, dense
from workloads import configs, Box, runs_from_mask, site_coords, site_linear_index, normalise_input


def _full_box(n, L):
    box = Box.centred(n, L)
    runs = runs_from_mask(np.ones(box.n, bool))
    lin = site_linear_index(box, runs)
    return box, runs, lin


def test_g0_fixed_point_is_top_eigenvector_of_step_operator():
    """With g = 0 one step is psi -> S psi / |S psi| with the symmetric
    S = P (I - dt/2 T~)^2 P, so the iteration converges to S's top eigenvector."""
    w = configs.small_shell(n=14, half_width=6.0, R0=3.0)
    lin = site_linear_index(w.box, w.runs)
    T = op.kinetic_direct(w.box.n, w.box.h, lin)
    dt = 0.02
    P = np.exp(-w.field * dt / 2)
    A = np.eye(lin.size) - (dt / 2) * T.toarray()
    S = np.diag(P) @ A @ A @ np.diag(P)
    ev, W = np.linalg.eigh(S)
    v = W[:, -1]
    gap = ev[-1] / ev[-2]
    steps = int(np.ceil(np.log(1e-13) / np.log(1 / gap)))
    psi, _ = itp.imaginary_time(T, w.psi0, w.field, 0.0, dt, w.box.dV, steps)
    c = np.vdot(v, psi)
    resid = psi - c * v
    assert np.linalg.norm(resid) <= 1e-10 * np.linalg.norm(psi)
    assert abs(ob.norm(psi, w.box.dV) - 1.0) < 1e-13


def test_harmonic_ground_energy_is_three_times_1d_eigenvalue():
    """Full box, V = r^2/2, g = 0: the 3D discrete ground energy separates into
    3 e1 with e1 the lowest eigenvalue of the 1D Dirichlet H (eigh); the
    split-step fixed point reaches it up to O(dt^2) (variational)."""
    box, runs, lin = _full_box(32, 8.0)
    T = op.kinetic_direct(box.n, box.h, lin)
    x, y, z = site_coords(box, runs)
    V = 0.5 * (x * x + y * y + z * z)
    xs = box.axis(0)
    H1 = -0.5 * op.second_difference_1d(32, box.h[0]).toarray() + np.diag(0.5 * xs * xs)
    e1 = np.linalg.eigvalsh(H1)[0]
    # approaches 3/2 - 3h^2/32 (the second-order FD correction), h = 0.5
    assert abs(3 * e1 - (1.5 - 3 * box.h[0] ** 2 / 32)) < 1e-3
    rng = np.random.default_rng(0)
    psi0 = np.exp(-(x * x + y * y + z * z) / 2) + 1e-3 * (rng.uniform(-1, 1, x.size) + 1j * rng.uniform(-1, 1, x.size))
    errs = []
    for dt in (0.02, 0.01):
        psi, _ = itp.imaginary_time(T, psi0, V, 0.0, dt, box.dV, int(25 / dt))
        _, E, mu = ob.energy_mu(T, psi, V, 0.0, box.dV)
        assert abs(E - mu) < 1e-12
        errs.append(E - 3 * e1)
    assert errs[1] > 0 and errs[1] < 1e-5
    assert 3.5 < errs[0] / errs[1] < 4.5      # O(dt^2)


@pytest.mark.slow
def test_thomas_fermi_limit_harmonic():
    """mu -> mu_TF = 1/2 (15 g / 4 pi)^(2/5) for a harmonic trap at large g (N = 1)."""
    box, runs, lin = _full_box(40, 8.0)
    T = op.kinetic_direct(box.n, box.h, lin)
    x, y, z = site_coords(box, runs)
    V = 0.5 * (x * x + y * y + z * z)
    rel = []
    for g in (1e2, 1e3, 1e4):
        mu_tf = 0.5 * (15 * g / (4 * np.pi)) ** 0.4
        psi0 = normalise_input((np.sqrt(np.maximum(mu_tf - V, 0) / g) + 1e-3).astype(complex), box.dV)
        psi, _ = itp.imaginary_time(T, psi0, V, g, 0.005, box.dV, 1000)
        _, E, mu = ob.energy_mu(T, psi, V, g, box.dV)
        rel.append((mu - mu_tf) / mu_tf)
    assert rel[0] > rel[1] > rel[2] > 0
    assert rel[2] < 0.03


def test_masked_equals_dense_when_mask_covers_box():
    w = configs.full_box_problem(n=8, half_width=2.0, g=10.0)
    lin = site_linear_index(w.box, w.runs)
    T = op.kinetic_kron(w.box.n, w.box.h, lin)
    psi, _ = itp.imaginary_time(T, w.psi0, w.field, w.g, 0.01, w.box.dV, 20)
    Vbox = w.field.reshape(w.box.n)
    ref = dense.dense_itp(w.box.n, w.box.h, w.extra["mask"], Vbox, w.psi0.reshape(w.box.n), w.g, 0.01, 20)
    assert np.linalg.norm(psi - ref.ravel()) <= 1e-13 * np.linalg.norm(ref)


def test_masked_equals_dense_projector_on_random_mask():
    w = configs.random_mask_problem(n=(6, 7, 5), density=0.55, seed=4, g=30.0)
    mask = w.extra["mask"]
    lin = site_linear_index(w.box, w.runs)
    T = op.kinetic_direct(w.box.n, w.box.h, lin)
    psi, _ = itp.imaginary_time(T, w.psi0, w.field, w.g, 0.005, w.box.dV, 15)
    Vbox = np.zeros(w.box.n)
    Vbox.ravel()[lin] = w.field
    p0 = np.zeros(w.box.n, complex)
    p0.ravel()[lin] = w.psi0
    ref = dense.dense_itp(w.box.n, w.box.h, mask, Vbox, p0, w.g, 0.005, 15).ravel()
    assert np.max(np.abs(ref[~mask.ravel()])) == 0.0
    assert np.linalg.norm(psi - ref[lin]) <= 1e-13 * np.linalg.norm(ref)


def test_observables_on_eigenvector():
    """g = 0: for an eigenvector of H~ = T~ + V~ the energy and mu equal its eigenvalue."""
    w = configs.random_mask_problem(n=(5, 6, 7), density=0.7, seed=9)
    lin = site_linear_index(w.box, w.runs)
    T = op.kinetic_direct(w.box.n, w.box.h, lin)
    H = T.toarray() + np.diag(w.field)
    ev, W = np.linalg.eigh(H)
    for idx in (0, 3, lin.size - 1):
        psi = W[:, idx] * (0.3 + 0.4j)
        N, E, mu = ob.energy_mu(T, psi, w.field, 0.0, w.box.dV)
        assert abs(N - 0.25 * w.box.dV) < 1e-15
        assert abs(E - ev[idx]) < 1e-12 * max(1.0, abs(ev[idx]))
        assert abs(mu - ev[idx]) < 1e-12 * max(1.0, abs(ev[idx]))
    # interaction term: for a constant |psi| the g-parts of E and mu are g/2 |psi|^2 and g |psi|^2
    psi = np.full(lin.size, 0.7 + 0.0j)
    _, E0, mu0 = ob.energy_mu(T, psi, w.field, 0.0, w.box.dV)
    _, E1, mu1 = ob.energy_mu(T, psi, w.field, 2.0, w.box.dV)
    assert abs((E1 - E0) - 0.49) < 1e-14 and abs((mu1 - mu0) - 0.98) < 1e-14


def test_real_start_stays_real_and_phase_is_carried():
    """Sec. II.A: with a real start, real V and real g every factor of one
    step (the diagonal half-steps and the Euler substeps with the real
    symmetric T~) is real, so psi stays real: the oracle's complex step on a
    real input leaves exactly zero imaginary parts.  The step is also
    equivariant under a global phase (it depends on psi only through psi and
    |psi|^2), so a start e^{i theta} x ends at e^{i theta} times the real
    result; a stray conjugation or a dropped imaginary term breaks this."""
    w = configs.random_mask_problem(n=(9, 8, 10), density=0.5, seed=5, g=30.0)
    lin = site_linear_index(w.box, w.runs)
    T = op.kinetic_direct(w.box.n, w.box.h, lin)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(lin.size)
    x /= np.sqrt(np.sum(x * x) * w.box.dV)
    dt = 1e-3
    out, _ = itp.imaginary_time(T, x.astype(complex), w.field, w.g, dt, w.box.dV, 12)
    assert np.all(out.imag == 0.0)
    ph = np.exp(0.7j)
    rot, _ = itp.imaginary_time(T, ph * x, w.field, w.g, dt, w.box.dV, 12)
    assert np.max(np.abs(rot - ph * out.real)) <= 1e-13 * np.max(np.abs(out))


def test_virial_theorem_of_the_interacting_harmonic_ground_state():
    """For V = r^2/2 the ground state of the GP energy satisfies the virial
    identity 2 E_kin - 2 E_pot + 3 E_int = 0 (scaling psi(x) -> l^{3/2}
    psi(l x) keeps the norm and leaves E stationary at l = 1).  E_kin and
    E_pot are computed here from their definitions; E_int is mu - E of the
    oracle's observables, so a wrong weight of the |psi|^4 term in E or mu,
    or of the kinetic term, breaks the identity by O(E).  The imaginary-time
    fixed point carries a residual linear in dt and the grid one of O(h^2)
    (measured: about 1.24 dt + 0.08 h^2), so the test halves dt, checks the
    residual falls, and bounds its dt -> 0 extrapolation."""
    box, runs, lin = _full_box(32, 4.8)
    T = op.kinetic_direct(box.n, box.h, lin)
    x, y, z = site_coords(box, runs)
    V = 0.5 * (x * x + y * y + z * z)
    g = 30.0
    psi0 = normalise_input(np.exp(-0.4 * (x * x + y * y + z * z)).astype(complex), box.dV)
    res = []
    for dt, steps in ((0.01, 1500), (0.005, 3000)):
        psi, _ = itp.imaginary_time(T, psi0, V, g, dt, box.dV, steps)
        N, E, mu = ob.energy_mu(T, psi, V, g, box.dV)
        e_kin = float(np.real(np.vdot(psi, op.apply(T, psi)))) * box.dV / N
        e_pot = float(np.sum(V * np.abs(psi) ** 2)) * box.dV / N
        e_int = mu - E
        assert abs(E - (e_kin + e_pot + e_int)) <= 1e-12 * E
        assert e_int > 0.1 * E                    # the interaction matters at this g
        res.append(2 * e_kin - 2 * e_pot + 3 * e_int)
    assert 0 < res[1] < res[0] < 0.01 * E
    assert abs(2 * res[1] - res[0]) <= 5e-3 * E   # the O(h^2) part, h = 0.3
