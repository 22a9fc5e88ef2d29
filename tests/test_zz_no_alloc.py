"""GPU test of the allocation-free real-time entry point, called through the
C ABI: two calls in a row (the second on a smaller grid) give exactly what
gpe_real_time gives with a caller work buffer, and a grid too large for the
library's static scratch is refused before anything runs."""
import ctypes as C

import numpy as np
import pytest

from workloads import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run_both(w, dtype, steps, integrator="rk4"):
    import torch
    from paper_2603_05447_amd import Grid, Potential, make_params, _lib
    lib = _lib.load()
    cdt = torch.complex128 if dtype == "c128" else torch.complex64
    rdt = torch.float64 if dtype == "c128" else torch.float32
    dt_ = _lib.GPE_C128 if dtype == "c128" else _lib.GPE_C64
    g = Grid.from_box(w.box, runs=w.runs, device=0)
    field = torch.tensor(w.field, dtype=rdt, device="cuda:0")
    pot = Potential.rf(field, w.omega, w.knot_t, w.knot_delta) if w.kind == "rf" else Potential.static(field)
    cp, keep = pot.as_c(dt_)
    prm = make_params(w.g, w.dt, integrator=integrator)
    a = torch.tensor(w.psi0, dtype=cdt, device="cuda:0")
    b = a.clone()
    mode = {"rk4": _lib.GPE_MODE_RT, "rkhe3": _lib.GPE_MODE_RT_RKHE3, "rkck": _lib.GPE_MODE_RT_RKCK}[integrator]
    nb = g.work_bytes(dt_, mode, steps)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    oa, ob = _lib.Obs(), _lib.Obs()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(lib.gpe_real_time(g.handle, dt_, a.data_ptr(), C.byref(cp), C.byref(prm), 0.0, steps,
                                 work.data_ptr(), nb, stream, C.byref(oa), None))
    _lib.check(lib.gpe_real_time_noalloc(g.handle, dt_, b.data_ptr(), C.byref(cp), C.byref(prm), 0.0, steps,
                                         stream, C.byref(ob), None))
    torch.cuda.synchronize()
    return a, b, oa, ob


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noalloc_equals_real_time_on_two_calls(dtype):
    import torch
    big = configs.small_rf_ramp(n=32, steps=20, g=300.0)
    small = configs.small_shell(n=16)
    for w, steps in ((big, 20), (small, 7)):
        a, b, oa, ob = _run_both(w, dtype, steps)
        print(f"{w.name} {dtype}: {w.n_active} sites, {steps} steps, identical "
              f"{bool(torch.equal(a, b))}", flush=True)
        assert torch.equal(a, b)
        assert (oa.norm, oa.energy, oa.mu) == (ob.norm, ob.energy, ob.mu)


def test_noalloc_other_integrators_and_size_limit():
    import torch
    from paper_2603_05447_amd import Grid, Potential, make_params, _lib
    w = configs.small_rf_ramp(n=24, steps=10, g=300.0)
    for integ in ("rkhe3", "rkck"):
        a, b, _, _ = _run_both(w, "c128", 5, integ)
        assert torch.equal(a, b), integ
    # a full 120^3 box needs 3 x 1.728M x 16 bytes > 64 MiB in complex128 RK4
    lib = _lib.load()
    assert lib.gpe_noalloc_scratch_bytes() == 64 << 20
    n = 120
    from workloads import Box
    b120 = Box.centred(n, 6.0)
    g = Grid.from_box(b120, mask=np.ones((n, n, n), bool), device=0)
    field = torch.zeros(g.n_active, dtype=torch.float64, device="cuda:0")
    psi = torch.zeros(g.n_active, dtype=torch.complex128, device="cuda:0")
    cp, keep = Potential.static(field).as_c(_lib.GPE_C128)
    prm = make_params(0.0, 1e-3)
    st = lib.gpe_real_time_noalloc(g.handle, _lib.GPE_C128, psi.data_ptr(), C.byref(cp), C.byref(prm), 0.0, 1,
                                   None, None, None)
    assert st == _lib.GPE_ERR_ARG and b"at most" in lib.gpe_last_error()
    # the same grid fits in complex64 (3 x 1.728M x 8 bytes = 41.5 MB)
    psi64 = torch.zeros(g.n_active, dtype=torch.complex64, device="cuda:0")
    f32 = torch.zeros(g.n_active, dtype=torch.float32, device="cuda:0")
    cp, keep = Potential.static(f32).as_c(_lib.GPE_C64)
    _lib.check(lib.gpe_real_time_noalloc(g.handle, _lib.GPE_C64, psi64.data_ptr(), C.byref(cp), C.byref(prm), 0.0,
                                         2, None, None, None))
    torch.cuda.synchronize()
    assert torch.count_nonzero(psi64).item() == 0
