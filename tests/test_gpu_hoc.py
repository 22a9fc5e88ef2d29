"""GPU parity of the 19-point higher-order compact stencil (App. B eq. (B2))
and of the cubic 27-point stencil through the C ABI against the oracle's
operators, for every path that applies T~: imaginary time (complex and real
state), real time with RK4 / RKHE3 / RKCK, observations, and the fidelity
gradient.

Tolerances: relative L2 <= 1e-10 (complex128), <= 1e-5 (complex64)."""
import numpy as np
import pytest

from oracle import itp, realtime as rt, observables as ob, tableau
from oracle import adjoint as adj
from oracle import operator as op
from workloads import configs, site_linear_index

from gpu_cases import Case, parity_err, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-10, "c64": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_05447_amd as p
    p.load_library()


def _hoc_case(w, dtype, points=19):
    c = Case(w, dtype)
    c.grid.set_stencil(points)
    assert c.grid.get_stencil() == points
    lin = site_linear_index(w.box, w.runs)
    c.T19 = (op.kinetic_direct_19 if points == 19 else op.kinetic_direct_27)(w.box.n, w.box.h, lin)
    return c


MAKERS = [lambda: configs.random_mask_problem(n=(12, 11, 13), density=0.5, seed=41, g=40.0, h=(0.5, 0.42, 0.37)),
          lambda: configs.small_shell(n=24)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("make", MAKERS, ids=["random-aniso", "shell24"])
def test_hoc_imag_time_matches_oracle(dtype, make):
    w = make()
    c = _hoc_case(w, dtype)
    psi = c.psi()
    obs = c.grid.imag_time(psi, c.pot, w.g, 2e-3, 20)
    ref, _ = itp.imaginary_time(c.T19, w.psi0, w.field, w.g, 2e-3, w.box.dV, 20)
    err = parity_err(psi.cpu().numpy(), ref)
    print(f"HOC ITP {w.name} {dtype}: parity error {err:.3e}", flush=True)
    assert err <= TOL[dtype]
    N, E, mu = ob.energy_mu(c.T19, ref, w.field, w.g, w.box.dV)
    assert abs(obs["energy"] - E) <= TOL[dtype] * abs(E) * 10
    assert abs(obs["mu"] - mu) <= TOL[dtype] * abs(mu) * 10


def test_hoc_real_state_imag_time_matches_oracle():
    import torch
    w = MAKERS[0]()
    c = _hoc_case(w, "c128")
    x = np.abs(w.psi0)
    x = x / np.sqrt(np.sum(x * x) * w.box.dV)
    psi = torch.tensor(x, dtype=torch.float64, device="cuda:0")
    c.grid.imag_time(psi, c.pot, w.g, 2e-3, 15, observe=False)
    ref, _ = itp.imaginary_time(c.T19, x.astype(complex), w.field, w.g, 2e-3, w.box.dV, 15)
    assert parity_err(psi.cpu().numpy(), ref.real) <= 1e-10


@pytest.mark.parametrize("integrator", ["rk4", "rkhe3", "rkck"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_hoc_real_time_matches_oracle(integrator, dtype):
    w = configs.small_rf_ramp(n=24, steps=20)
    c = _hoc_case(w, dtype)
    psi = c.psi()
    c.grid.real_time(psi, c.pot, w.g, 1e-3, 20, t0=0.003, integrator=integrator, observe=False)
    if integrator == "rk4":
        ref = rt.real_time(c.T19, w.psi0, c.opot, w.g, 1e-3, 0.003, 20)
    else:
        A, b = (tableau.heun3 if integrator == "rkhe3" else tableau.cash_karp5)()
        ref = rt.real_time_tableau(c.T19, w.psi0, c.opot, w.g, 1e-3, 0.003, 20, A, b)
    err = parity_err(psi.cpu().numpy(), ref)
    print(f"HOC {integrator} {dtype}: parity error {err:.3e}", flush=True)
    assert err <= TOL[dtype]
    # the 7-point path really differs from the 19-point one here
    ref7 = rt.real_time(c.T, w.psi0, c.opot, w.g, 1e-3, 0.003, 20)
    assert rel_l2(ref7, ref) > 1e3 * TOL["c128"]


def test_hoc_fidelity_gradient_matches_oracle_adjoint():
    w = configs.small_rf_ramp(n=20, steps=16, g=250.0, n_knots=5)
    c = _hoc_case(w, "c128")
    rng = np.random.default_rng(3)
    tgt = w.psi0 * np.exp(1j * rng.uniform(0, 0.3, w.n_active))
    loss, grad = c.grid.fidelity_grad(c.psi(), c.psi(tgt), c.pot, w.g, w.dt, w.steps)
    oloss, ograd, _ = adj.fidelity_grad(c.T19, c.opot, w.g, w.dt, 0.0, w.steps, w.psi0, tgt, w.box.dV)
    assert abs(loss - oloss) <= 1e-10 * max(abs(oloss), 1e-3)
    assert np.max(np.abs(grad - ograd)) <= 1e-9 * np.max(np.abs(ograd))


def test_hoc_switch_back_and_stability_bound():
    from paper_2603_05447_amd import GPEError, _lib
    w = MAKERS[0]()
    c = _hoc_case(w, "c128")
    with pytest.raises(GPEError):
        c.grid.set_stencil(27)
    # the 19-point operator's Gershgorin bound is below the 7-point one: a dt
    # just above 4/lambda_7 passes the imaginary-time check with 19 points
    h2 = [v * v for v in w.box.h]
    lam7 = 2 * sum(1 / v for v in h2)
    dt = 4.2 / lam7
    c.grid.imag_time(c.psi(), c.pot, w.g, dt, 1, observe=False, check_stability=True)
    c.grid.set_stencil(7)
    with pytest.raises(GPEError) as e:
        c.grid.imag_time(c.psi(), c.pot, w.g, dt, 1, observe=False, check_stability=True)
    assert e.value.status == _lib.GPE_ERR_UNSTABLE
    psi = c.psi()
    c.grid.real_time(psi, c.pot, w.g, 1e-3, 5, observe=False)
    ref = rt.real_time(c.T, w.psi0, c.opot, w.g, 1e-3, 0.0, 5)
    assert parity_err(psi.cpu().numpy(), ref) <= 1e-10


ISO = [lambda: configs.random_mask_problem(n=(12, 11, 13), density=0.5, seed=43, g=40.0, h=(0.42, 0.42, 0.42)),
       lambda: configs.small_shell(n=24)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("make", ISO, ids=["random-iso", "shell24"])
def test_27pt_imag_time_matches_oracle(dtype, make):
    w = make()
    c = _hoc_case(w, dtype, 27)
    psi = c.psi()
    obs = c.grid.imag_time(psi, c.pot, w.g, 2e-3, 20)
    ref, _ = itp.imaginary_time(c.T19, w.psi0, w.field, w.g, 2e-3, w.box.dV, 20)
    err = parity_err(psi.cpu().numpy(), ref)
    print(f"27pt ITP {w.name} {dtype}: parity error {err:.3e}", flush=True)
    assert err <= TOL[dtype]
    N, E, mu = ob.energy_mu(c.T19, ref, w.field, w.g, w.box.dV)
    assert abs(obs["energy"] - E) <= TOL[dtype] * abs(E) * 10


@pytest.mark.parametrize("integrator", ["rk4", "rkck"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_27pt_real_time_matches_oracle(integrator, dtype):
    w = configs.small_rf_ramp(n=24, steps=20)
    c = _hoc_case(w, dtype, 27)
    psi = c.psi()
    c.grid.real_time(psi, c.pot, w.g, 1e-3, 20, t0=0.003, integrator=integrator, observe=False)
    if integrator == "rk4":
        ref = rt.real_time(c.T19, w.psi0, c.opot, w.g, 1e-3, 0.003, 20)
    else:
        A, b = tableau.cash_karp5()
        ref = rt.real_time_tableau(c.T19, w.psi0, c.opot, w.g, 1e-3, 0.003, 20, A, b)
    err = parity_err(psi.cpu().numpy(), ref)
    print(f"27pt {integrator} {dtype}: parity error {err:.3e}", flush=True)
    assert err <= TOL[dtype]


def test_27pt_needs_equal_spacings():
    from paper_2603_05447_amd import GPEError, _lib
    w = MAKERS[0]()             # anisotropic spacings
    c = Case(w, "c128")
    with pytest.raises(GPEError) as e:
        c.grid.set_stencil(27)
    assert e.value.status == _lib.GPE_ERR_ARG
    assert c.grid.get_stencil() == 7
