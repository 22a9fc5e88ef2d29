"""GPU parity of the staged-ramp pieces (Sec. V): the stage potential
interpolated in time between two arrays (GPE_POT_LERP), post-selection on the
device (gpe_grid_create_threshold), the carry-over of psi between grids
(gpe_remap, bit-exact), the real-field pack, and a whole staged ramp with
re-post-selection at every stage against the oracle doing the same steps.

Tolerances: relative L2 <= 1e-10 (complex128), <= 1e-5 (complex64);
integer and data-movement results bit-exact."""
import numpy as np
import pytest

from oracle import itp, realtime as rt, restage
from oracle import operator as op
from workloads import Box, configs, runs_from_mask, site_linear_index

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


def _t(a, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_lerp_stage_real_time_matches_oracle(dtype):
    import torch
    from paper_2603_05447_amd import Potential
    w = configs.random_mask_problem(n=(12, 11, 13), density=0.45, seed=31, g=40.0)
    c = Case(w, dtype)
    rng = np.random.default_rng(5)
    Vb = w.field + rng.uniform(-2.0, 3.0, w.n_active)
    # the run starts before the stage and ends after it: both clamps are used
    ta, tb, t0, dt, steps = 0.004, 0.02, 0.0, 1e-3, 30
    pot = Potential.lerp(c.field, _t(Vb, c.rdt), ta, tb)
    psi = c.psi()
    obs = c.grid.real_time(psi, pot, w.g, dt, steps, t0=t0)
    opot = restage.LerpPotential(w.field, Vb, ta, tb)
    ref = rt.real_time(c.T, w.psi0, opot, w.g, dt, t0, steps)
    assert parity_err(psi.cpu().numpy(), ref) <= TOL[dtype]
    from oracle import observables as ob
    N, E, mu = ob.energy_mu(c.T, ref, opot(t0 + steps * dt), w.g, w.box.dV)
    assert abs(obs["energy"] - E) <= TOL[dtype] * abs(E) * 10
    # imaginary time takes V at t = 0: the start array before the stage
    p2 = c.psi()
    c.grid.imag_time(p2, pot, w.g, 2e-3, 10, observe=False)
    r2, _ = itp.imaginary_time(c.T, w.psi0, opot(0.0), w.g, 2e-3, w.box.dV, 10)
    assert parity_err(p2.cpu().numpy(), r2) <= TOL[dtype]


@pytest.mark.parametrize("rdt", ["f64", "f32"])
def test_threshold_grid_matches_oracle_mask(rdt):
    import torch
    from paper_2603_05447_amd import Grid
    s = configs.staged_rf_shells(n=20)
    tdt = torch.float64 if rdt == "f64" else torch.float32
    npdt = np.float64 if rdt == "f64" else np.float32
    Va, Vb = s.fields[0].astype(npdt), s.fields[2].astype(npdt)
    cut = 12.25                       # exactly representable in float32
    g = Grid.from_threshold(s.box.n, s.box.h, s.box.x0, _t(Va, tdt), _t(Vb, tdt), cut, device=0)
    want = restage.post_select(Va, Vb, cut)
    got = site_linear_index(s.box, g.runs()[:, :4])
    assert np.array_equal(got, np.flatnonzero(want.ravel()))
    g1 = Grid.from_threshold(s.box.n, s.box.h, s.box.x0, _t(Va, tdt), None, cut, device=0)
    assert np.array_equal(site_linear_index(s.box, g1.runs()[:, :4]), np.flatnonzero((Va < cut).ravel()))


@pytest.mark.parametrize("n2", [1, 63, 64, 128, 150, 300])
def test_threshold_runs_cross_the_64_point_steps(n2):
    """Runs that start at k = 0, end at k = n2, cross multiples of 64, and
    single-point runs: the device-built run table equals the runs of the
    dense selection."""
    import torch
    from paper_2603_05447_amd import Grid
    rng = np.random.default_rng(n2)
    n = (5, 6, n2)
    va = rng.uniform(0.0, 1.0, n)
    vb = rng.uniform(0.0, 1.0, n)
    # long stretches in some columns, isolated points in others
    va[0, :, :] = 0.0
    va[1, 2, ::2] = 2.0
    va[2, :, n2 // 2:] = 0.1
    vb[2, :, :] = 5.0
    cut = 0.3
    box = Box(n, (0.1, 0.1, 0.1), (0.0, 0.0, 0.0))
    g = Grid.from_threshold(n, box.h, box.x0, torch.tensor(va, device="cuda:0"), torch.tensor(vb, device="cuda:0"),
                            cut, device=0)
    want = runs_from_mask(np.minimum(va, vb) < cut)
    assert np.array_equal(g.runs()[:, :4], want)


def test_threshold_with_nothing_selected_is_an_argument_error():
    import torch
    from paper_2603_05447_amd import Grid, GPEError, _lib
    n = (4, 5, 70)
    va = torch.ones(n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(GPEError) as e:
        Grid.from_threshold(n, (0.1, 0.1, 0.1), (0.0, 0.0, 0.0), va, None, 0.5, device=0)
    assert e.value.status == _lib.GPE_ERR_ARG
    with pytest.raises(GPEError) as e:       # NaN never passes the cut
        Grid.from_threshold(n, (0.1, 0.1, 0.1), (0.0, 0.0, 0.0), va * float("nan"), None, 2.0, device=0)
    assert e.value.status == _lib.GPE_ERR_ARG


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_remap_is_exact(dtype):
    import torch
    from paper_2603_05447_amd import Grid
    rng = np.random.default_rng(11)
    box = Box.centred((9, 7, 11), 3.0)
    ma = rng.uniform(size=box.n) < 0.55
    mb = rng.uniform(size=box.n) < 0.45
    ga = Grid.from_box(box, mask=ma, device=0)
    gb = Grid.from_box(box, mask=mb, device=0)
    la = site_linear_index(box, runs_from_mask(ma))
    lb = site_linear_index(box, runs_from_mask(mb))
    cdt = torch.complex128 if dtype == "c128" else torch.complex64
    npc = np.complex128 if dtype == "c128" else np.complex64
    psi = (rng.standard_normal(la.size) + 1j * rng.standard_normal(la.size)).astype(npc)
    out = gb.remap_from(ga, _t(psi, cdt))
    assert np.array_equal(out.cpu().numpy(), restage.remap(psi, la, lb))
    back = ga.remap_from(gb, out)
    assert np.array_equal(back.cpu().numpy(), restage.remap(restage.remap(psi, la, lb), lb, la))


def test_remap_and_pack_argument_checks():
    import torch
    from paper_2603_05447_amd import Grid, GPEError, _lib
    rng = np.random.default_rng(12)
    b1, b2 = Box.centred((6, 6, 6), 3.0), Box.centred((6, 6, 7), 3.0)
    g1 = Grid.from_box(b1, mask=rng.uniform(size=b1.n) < 0.5, device=0)
    g2 = Grid.from_box(b2, mask=rng.uniform(size=b2.n) < 0.5, device=0)
    x = torch.zeros(g1.n_active, dtype=torch.complex128, device="cuda:0")
    with pytest.raises(GPEError) as e:
        g2.remap_from(g1, x)
    assert e.value.status == _lib.GPE_ERR_ARG
    with pytest.raises(GPEError) as e:
        g1.remap_from(g1, x, out=x)
    assert e.value.status == _lib.GPE_ERR_ARG
    with pytest.raises(ValueError):
        g1.pack(torch.zeros(10, dtype=torch.float64, device="cuda:0"))
    # real pack is the box gather
    V = rng.uniform(size=b1.n)
    lin = site_linear_index(b1, g1.runs()[:, :4])
    assert np.array_equal(g1.pack(_t(V, torch.float64)).cpu().numpy(), V.ravel()[lin])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_staged_ramp_matches_oracle(dtype):
    """Three stages, each re-post-selected from min(V_i, V_{i+1}) < 5
    max(mu_i, mu_{i+1}), psi carried over, then evolved with the
    interpolated potential; the oracle takes the same steps."""
    import torch
    from paper_2603_05447_amd import Grid, staged_ramp
    s = configs.staged_rf_shells(n=20)
    box = s.box
    cdt = torch.complex128 if dtype == "c128" else torch.complex64
    rdt = torch.float64 if dtype == "c128" else torch.float32
    full = np.ones(box.n, bool)
    g0 = Grid.from_box(box, mask=full, device=0)
    psi = _t(s.psi0_box.ravel(), cdt)
    fields = [_t(f, rdt) for f in s.fields]
    g, out, recs = staged_ramp(g0, psi, fields, s.mus, s.g, s.dt, s.steps_per_stage)
    # oracle
    lin = np.arange(full.size)
    y = s.psi0_box.ravel().astype(np.complex128)
    for i in range(len(s.fields) - 1):
        cut = restage.stage_cutoff(s.mus[i], s.mus[i + 1])
        m = restage.post_select(s.fields[i], s.fields[i + 1], cut)
        new = np.flatnonzero(m.ravel())
        y = restage.remap(y, lin, new)
        lin = new
        T = op.kinetic_direct(box.n, box.h, lin)
        ta = i * s.steps_per_stage * s.dt
        pot = restage.LerpPotential(s.fields[i].ravel()[lin], s.fields[i + 1].ravel()[lin], ta,
                                    ta + s.steps_per_stage * s.dt)
        y = rt.real_time(T, y, pot, s.g, s.dt, ta, s.steps_per_stage)
        assert recs[i]["n_active"] == lin.size
    assert np.array_equal(site_linear_index(box, g.runs()[:, :4]), lin)
    assert parity_err(out.cpu().numpy(), y) <= TOL[dtype]
    assert recs[0]["norm_after_remap"] < 1.0          # the first selection drops the tail outside the shell
