"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle,
element by element on the same seeded inputs.

Tolerances (relative L2 over all sites): complex128 <= 1e-10; complex64
<= 1e-5 over short horizons (FP32 stencil, FP64 reductions)."""
import numpy as np
import pytest

from oracle import itp, realtime as rt, observables as ob
from workloads import configs

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


def _print(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("make", [lambda: configs.small_shell(n=24),
                                  lambda: configs.random_mask_problem(n=(12, 11, 13), density=0.45, seed=31, g=40.0)],
                         ids=["shell24", "random"])
def test_imag_time_matches_oracle(dtype, make):
    w = make()
    c = Case(w, dtype)
    _print(f"ITP {w.name} n={w.n_active} {dtype}")
    steps, dt = 25, 2e-3
    psi = c.psi()
    obs = c.grid.imag_time(psi, c.pot, w.g, dt, steps)
    ref, _ = itp.imaginary_time(c.T, w.psi0, w.field, w.g, dt, w.box.dV, steps)
    err = parity_err(psi.cpu().numpy(), ref)
    _print(f"  parity error = {err:.3e}")
    assert err <= TOL[dtype]
    N, E, mu = ob.energy_mu(c.T, ref, w.field, w.g, w.box.dV)
    assert abs(obs["norm"] - 1.0) < 1e-12 if dtype == "c128" else abs(obs["norm"] - 1.0) < 1e-6
    assert abs(obs["energy"] - E) <= TOL[dtype] * abs(E) * 10
    assert abs(obs["mu"] - mu) <= TOL[dtype] * abs(mu) * 10


def test_c1_imag_time_500_steps_fp64():
    """C1: 64^3 shell, g = 100, 500 imaginary-time steps, dt = 1e-3, complex128."""
    w = configs.c1()
    c = Case(w, "c128")
    psi = c.psi()
    hist = None
    import torch
    hist = torch.zeros((5, 3), dtype=torch.float64, device=c.dev)
    obs = c.grid.imag_time(psi, c.pot, w.g, w.dt, w.steps, obs_every=100, history=hist)
    ohist = []
    ref, ohist = itp.imaginary_time(c.T, w.psi0, w.field, w.g, w.dt, w.box.dV, w.steps, observe_every=100)
    err = parity_err(psi.cpu().numpy(), ref)
    _print(f"C1 ITP 500 steps: parity error = {err:.3e}, E = {obs['energy']:.12f}")
    assert err <= 1e-10
    h = hist.cpu().numpy()
    for k, row in enumerate(ohist):
        assert abs(h[k, 0] - row[1]) < 1e-12
        assert abs(h[k, 1] - row[2]) <= 1e-10 * abs(row[2])
        assert abs(h[k, 2] - row[3]) <= 1e-10 * abs(row[3])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("make", [lambda: configs.small_rf_ramp(n=28, steps=30),
                                  lambda: configs.small_shell(n=24)], ids=["rframp28", "shell24"])
def test_real_time_matches_oracle(dtype, make):
    w = make()
    c = Case(w, dtype)
    steps, dt = 30, 1e-3
    _print(f"RK4 {w.name} n={w.n_active} {dtype}")
    psi = c.psi()
    obs = c.grid.real_time(psi, c.pot, w.g, dt, steps, t0=0.005)
    ref = rt.real_time(c.T, w.psi0, c.opot, w.g, dt, 0.005, steps)
    err = parity_err(psi.cpu().numpy(), ref)
    _print(f"  parity error = {err:.3e}")
    assert err <= TOL[dtype]
    N, E, mu = ob.energy_mu(c.T, ref, c.opot(0.005 + steps * dt), w.g, w.box.dV)
    assert abs(obs["norm"] - N) <= TOL[dtype] * N * 10
    assert abs(obs["energy"] - E) <= TOL[dtype] * abs(E) * 10


def test_real_time_history_matches_oracle():
    import torch
    w = configs.small_rf_ramp(n=24, steps=20)
    c = Case(w, "c128")
    psi = c.psi()
    hist = torch.zeros((4, 3), dtype=torch.float64, device=c.dev)
    c.grid.real_time(psi, c.pot, w.g, 1e-3, 20, t0=0.0, obs_every=5, history=hist)
    rows = []
    rt.real_time(c.T, w.psi0, c.opot, w.g, 1e-3, 0.0, 20,
                 observe=lambda n, t, y: rows.append(ob.energy_mu(c.T, y, c.opot(t), w.g, w.box.dV)), observe_every=5)
    h = hist.cpu().numpy()
    for k, (N, E, mu) in enumerate(rows):
        assert abs(h[k, 0] - N) <= 1e-12 * N
        assert abs(h[k, 1] - E) <= 1e-10 * abs(E)
        assert abs(h[k, 2] - mu) <= 1e-10 * abs(mu)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_observe_and_overlap(dtype):
    w = configs.small_rf_ramp(n=24)
    c = Case(w, dtype)
    rng = np.random.default_rng(8)
    other = w.psi0 * np.exp(1j * rng.uniform(0, 1, w.n_active))
    psi, b = c.psi(), c.psi(other)
    t = 0.013
    o = c.grid.observe(psi, c.pot, t, w.g)
    N, E, mu = ob.energy_mu(c.T, w.psi0, c.opot(t), w.g, w.box.dV)
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert abs(o["norm"] - N) <= tol * N and abs(o["energy"] - E) <= tol * abs(E) and abs(o["mu"] - mu) <= tol * abs(mu)
    ov = c.grid.overlap(psi, b)
    ref = ob.overlap(w.psi0, other, w.box.dV)
    assert abs(ov - ref) <= tol * abs(ref)


def test_every_launch_config_gives_the_same_result():
    from paper_2603_05447_amd import config_count
    w = configs.small_shell(n=24)
    base = None
    for k in range(config_count()):
        c = Case(w, "c128", config=k)
        psi = c.psi()
        c.grid.imag_time(psi, c.pot, w.g, 2e-3, 10, observe=False)
        c.grid.real_time(psi, c.pot, w.g, 1e-3, 10, observe=False)
        out = psi.cpu().numpy()
        if base is None:
            base = out
        else:
            assert parity_err(out, base) <= 1e-13, k


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_every_launch_config_matches_the_oracle_on_a_fragmented_mask(dtype):
    """Every launch variant (64 to 1024 lanes, 1 to 8 sites per lane, with and
    without LDS staging, every chunk order) against the oracle on a random
    mask whose chunks are cut at the 255-segment limit and end in ragged
    tails: imaginary time, then real time from its result."""
    from paper_2603_05447_amd import config_count
    w = configs.random_mask_problem(n=(18, 20, 22), density=0.5, seed=12)
    c0 = Case(w, dtype)
    ref, _ = itp.imaginary_time(c0.T, w.psi0, w.field, w.g, 2e-3, w.box.dV, 4)
    ref = rt.real_time(c0.T, ref, c0.opot, w.g, 1e-3, 0.0, 4)
    for k in range(config_count()):
        c = Case(w, dtype, config=k)
        psi = c.psi()
        c.grid.imag_time(psi, c.pot, w.g, 2e-3, 4, observe=False)
        c.grid.real_time(psi, c.pot, w.g, 1e-3, 4, observe=False)
        err = parity_err(psi.cpu().numpy(), ref)
        assert err <= TOL[dtype], (k, err)


@pytest.mark.parametrize("real", [False, True])
def test_small_grid_scale_formed_in_pass1_equals_the_finalize_path(real):
    """On small grids pass 1 forms the renormalisation scale from pass 2's
    norm partials (no finalize launch); a run with an observation history
    keeps the finalize.  Both give the same state to rounding."""
    import torch
    w = configs.small_shell(n=24)
    c = Case(w, "c128")
    a, b = c.psi(), c.psi()
    if real:
        a, b = a.real.contiguous(), b.real.contiguous()
    c.grid.imag_time(a, c.pot, w.g, 2e-3, 30, observe=False)
    hist = torch.zeros((1, 3), dtype=torch.float64, device="cuda:0")
    c.grid.imag_time(b, c.pot, w.g, 2e-3, 30, obs_every=30, history=hist, observe=False)
    assert parity_err(a.cpu().numpy(), b.cpu().numpy()) <= 1e-13


def test_imaginary_time_on_a_grid_of_many_chunks():
    """Grids of more than 1024 chunks renormalise through the finalize kernel
    after every step (smaller ones form the scale inside pass 1): 10
    imaginary-time steps of the downscaled C5 shell (931,864 sites, 1,821
    chunks) against the oracle, the returned norm, and two runs bitwise
    equal."""
    import torch
    w = configs.c5_subdomain(8)
    c = Case(w, "c128")
    V = np.sqrt((w.field - w.knot_delta[0]) ** 2 + w.omega ** 2)
    from paper_2603_05447_amd import Potential
    pot = Potential.static(torch.tensor(V, dtype=torch.float64, device="cuda:0"))
    a, b = c.psi(), c.psi()
    oa = c.grid.imag_time(a, pot, w.g, w.dt, 10)
    c.grid.imag_time(b, pot, w.g, w.dt, 10, observe=False)
    assert torch.equal(a, b)
    ref, _ = itp.imaginary_time(c.T, w.psi0, V, w.g, w.dt, w.box.dV, 10)
    err = parity_err(a.cpu().numpy(), ref)
    _print(f"many-chunk imaginary time, {w.n_active} sites: parity error {err:.3e}, norm {oa['norm']:.15f}")
    assert err <= 1e-10
    assert abs(oa["norm"] - 1.0) <= 1e-12


def test_stream_copy_reference_kernel():
    import torch
    from paper_2603_05447_amd import GPEError, _lib, stream_copy
    x = torch.randint(0, 256, (16 * 100_003,), dtype=torch.uint8, device="cuda:0")
    y = torch.zeros_like(x)
    stream_copy(x, y)
    assert torch.equal(x, y)
    for src, dst in ((x[:20], y), (x[1:17], y), (x[:64], x[32:96])):   # size, alignment, overlap
        with pytest.raises(GPEError) as e:
            stream_copy(src, dst)
        assert e.value.status == _lib.GPE_ERR_ARG


def test_runs_are_bitwise_reproducible():
    w = configs.small_rf_ramp(n=28)
    outs = []
    for _ in range(2):
        c = Case(w, "c128")
        psi = c.psi()
        c.grid.imag_time(psi, c.pot, w.g, 2e-3, 10, observe=False)
        c.grid.real_time(psi, c.pot, w.g, 1e-3, 10, observe=False)
        outs.append(psi.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_pack_unpack_roundtrip(dtype):
    import torch
    w = configs.random_mask_problem(n=(9, 10, 11), density=0.5, seed=4)
    c = Case(w, dtype)
    psi = c.psi()
    box = c.grid.unpack(psi)
    mask = w.extra["mask"]
    b = box.cpu().numpy()
    assert np.all(b[~mask] == 0)
    assert np.array_equal(b[mask], psi.cpu().numpy())
    back = c.grid.pack(box)
    assert torch.equal(back, psi)


def test_zero_steps_and_single_site():
    w = configs.small_shell(n=16)
    c = Case(w, "c128")
    psi = c.psi()
    c.grid.imag_time(psi, c.pot, w.g, 1e-3, 0, observe=False)
    c.grid.real_time(psi, c.pot, w.g, 1e-3, 0, observe=False)
    assert np.array_equal(psi.cpu().numpy(), w.psi0)
    # a single active site: T~ is the diagonal 1/hx^2 + 1/hy^2 + 1/hz^2
    from workloads import Box
    from workloads.configs import Workload
    box = Box((3, 3, 3), (0.5, 0.5, 0.5), (0.0, 0.0, 0.0))
    w1 = Workload("single", box, np.array([[1, 1, 1, 2]], np.int64), np.array([0.3]), "static", g=2.0,
                  psi0=np.array([0.7 + 0.1j]) / np.sqrt(0.5 * 0.125))
    c1 = Case(w1, "c128")
    p = c1.psi()
    c1.grid.real_time(p, c1.pot, w1.g, 1e-2, 7, observe=False)
    ref = rt.real_time(c1.T, w1.psi0, c1.opot, w1.g, 1e-2, 0.0, 7)
    assert parity_err(p.cpu().numpy(), ref) <= 1e-14


def test_stability_bound_and_nonfinite_watchdog():
    from paper_2603_05447_amd import GPEError, _lib
    w = configs.small_shell(n=16)
    c = Case(w, "c128")
    psi = c.psi()
    lam_t = 2 * sum(1 / h ** 2 for h in w.box.h)
    with pytest.raises(GPEError) as e:
        c.grid.imag_time(psi, c.pot, w.g, 4.5 / lam_t, 3, check_stability=True)
    assert e.value.status == _lib.GPE_ERR_UNSTABLE
    with pytest.raises(GPEError) as e:
        c.grid.real_time(psi, c.pot, w.g, 3.0 / lam_t, 3, check_stability=True)
    assert e.value.status == _lib.GPE_ERR_UNSTABLE
    assert np.array_equal(psi.cpu().numpy(), w.psi0)     # nothing ran
    # an all-zero state cannot be renormalised: the norm observed is NaN
    z = c.psi(np.zeros(w.n_active, complex))
    with pytest.raises(GPEError) as e:
        c.grid.imag_time(z, c.pot, w.g, 1e-3, 2)
    assert e.value.status == _lib.GPE_ERR_NONFINITE


def test_bad_arguments_are_rejected():
    import torch
    from paper_2603_05447_amd import GPEError, _lib
    w = configs.small_shell(n=16)
    c = Case(w, "c128")
    psi = c.psi()
    with pytest.raises(TypeError):
        c.grid.imag_time(psi, type(c.pot).static(c.field.float()), w.g, 1e-3, 1)
    with pytest.raises(GPEError) as e:
        c.grid.real_time(psi, c.pot, w.g, -1e-3, 1)
    assert e.value.status == _lib.GPE_ERR_ARG
    bad = type(c.pot).rf(c.field, 2.0, [0.0, 0.0], [1.0, 2.0])
    with pytest.raises(GPEError) as e:
        c.grid.real_time(psi, bad, w.g, 1e-3, 1)
    assert e.value.status == _lib.GPE_ERR_ARG
