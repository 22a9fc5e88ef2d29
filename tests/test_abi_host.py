"""Host-side tests of the C ABI library (no GPU needed): it loads, exports
every symbol include/gpe.h declares, and builds the compact layout (runs,
segments, lateral offsets) exactly (bit-exact integer work)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from workloads import configs, Box, runs_from_mask, site_ijk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpe.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2603_05447_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libgpe.so is not built (run __graft_entry__.build())")
    return _lib.load()


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gpe_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol(lib):
    from paper_2603_05447_amd import _lib
    names = declared_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, f"{n} has no ctypes signature"
    assert lib.gpe_abi_version() == 4
    assert lib.gpe_config_count() >= 6


def test_launch_variant_table_spans_the_tuning_space(lib):
    """The tuner's search space: 64 to 1024 lanes, 1 to 8 sites per lane, LDS
    staging on and off; every shape holds at least 256 sites per chunk."""
    from paper_2603_05447_amd import config_describe
    ds = [config_describe(k) for k in range(lib.gpe_config_count())]
    assert {d["block"] for d in ds} == {64, 128, 256, 512, 1024}
    assert {d["sites_per_lane"] for d in ds} == {1, 2, 4, 8}
    assert {d["lds_stage"] for d in ds} == {0, 1}
    assert all(d["block"] * d["sites_per_lane"] >= 256 for d in ds)
    assert ds[0] == {"block": 256, "sites_per_lane": 2, "xcd_map": 4, "rk_scheme": 1, "nontemporal": 1,
                     "lds_stage": 1}
    assert len({tuple(d.values()) for d in ds}) == len(ds)


def _expected_neighbours(box, runs):
    """Brute force: dense box -> compact index map; per site the compact index
    of its 6 neighbours (-1 outside the active set or the box)."""
    n0, n1, n2 = box.n
    idx = -np.ones(box.n, np.int64)
    i, j, k = site_ijk(runs)
    idx[i, j, k] = np.arange(i.size)
    out = -np.ones((i.size, 6), np.int64)
    for d, (di, dj, dk) in enumerate(((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))):
        a, b, c = i + di, j + dj, k + dk
        ok = (a >= 0) & (a < n0) & (b >= 0) & (b < n1) & (c >= 0) & (c < n2)
        out[ok, d] = idx[a[ok], b[ok], c[ok]]
    return out


def _neighbours_from_segments(segs, n_active):
    out = -np.ones((n_active, 6), np.int64)
    covered = np.zeros(n_active, np.int64)
    for start, length, flags, xm, xp, ym, yp, _ in segs:
        s = np.arange(start, start + length)
        covered[s] += 1
        for d, off in enumerate((xm, xp, ym, yp)):
            if off != 0:
                out[s, d] = s + off
        zm = s - 1
        zp = s + 1
        if flags & 1:
            zm[0] = -1
        if flags & 2:
            zp[-1] = -1
        out[s, 4] = zm
        out[s, 5] = zp
    assert np.all(covered == 1), "segments must tile the active sites exactly once"
    return out


def _host_grid(box, runs=None, mask=None):
    from paper_2603_05447_amd import Grid
    return Grid(box.n, box.h, box.x0, runs=runs, mask=mask, device=-1)


CASES = [
    ("random sparse", lambda: configs.random_mask_problem(n=(9, 8, 11), density=0.25, seed=1)),
    ("random dense", lambda: configs.random_mask_problem(n=(7, 10, 6), density=0.85, seed=2)),
    ("shell", lambda: configs.small_shell(n=20)),
    ("full box", lambda: configs.full_box_problem(n=6)),
    ("rf ramp", lambda: configs.small_rf_ramp(n=24)),
]


@pytest.mark.parametrize("name,make", CASES)
def test_segments_reproduce_brute_force_neighbours(lib, name, make):
    w = make()
    g = _host_grid(w.box, runs=w.runs)
    assert g.n_active == w.n_active
    segs = g.segments()
    got = _neighbours_from_segments(segs, g.n_active)
    ref = _expected_neighbours(w.box, w.runs)
    assert np.array_equal(got, ref)
    # runs come back in the same order with prefix-sum starts
    r = g.runs()
    assert np.array_equal(r[:, :4], w.runs)
    lens = w.runs[:, 3] - w.runs[:, 2]
    assert np.array_equal(r[:, 4], np.concatenate([[0], np.cumsum(lens)[:-1]]))


HOC_TAPS = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (-1, 0, -1), (-1, 0, 1), (1, 0, -1), (1, 0, 1),
            (0, -1, -1), (0, -1, 1), (0, 1, -1), (0, 1, 1), (-1, -1, 0), (-1, 1, 0), (1, -1, 0), (1, 1, 0),
            (-1, -1, -1), (-1, -1, 1), (-1, 1, -1), (-1, 1, 1), (1, -1, -1), (1, -1, 1), (1, 1, -1), (1, 1, 1))


@pytest.mark.parametrize("points", [19, 27])
@pytest.mark.parametrize("name,make", CASES)
def test_hoc_segments_reproduce_brute_force_taps(lib, name, make, points):
    """The 19/27-point tables: every active site's 16/24 lateral taps (and
    the run-end flags for k+-1) match a dense box lookup exactly."""
    w = make()
    g = _host_grid(w.box, runs=w.runs)
    segs = g.hoc_segments(points)
    ntap = 16 if points == 19 else 24
    n0, n1, n2 = w.box.n
    idx = -np.ones(w.box.n, np.int64)
    i, j, k = site_ijk(w.runs)
    idx[i, j, k] = np.arange(i.size)
    want = -np.ones((i.size, ntap), np.int64)
    for t, (di, dj, dk) in enumerate(HOC_TAPS[:ntap]):
        a, b, c = i + di, j + dj, k + dk
        ok = (a >= 0) & (a < n0) & (b >= 0) & (b < n1) & (c >= 0) & (c < n2)
        want[ok, t] = idx[a[ok], b[ok], c[ok]]
    got = -np.ones_like(want)
    covered = np.zeros(i.size, np.int64)
    zgot = -np.ones((i.size, 2), np.int64)
    for row in segs:
        start, length, flags = row[0], row[1], row[2]
        s = np.arange(start, start + length)
        covered[s] += 1
        for t in range(ntap):
            if row[3 + t] != 0:
                got[s, t] = s + row[3 + t]
        zm, zp = s - 1, s + 1
        if flags & 1:
            zm[0] = -1
        if flags & 2:
            zp[-1] = -1
        zgot[s, 0], zgot[s, 1] = zm, zp
    assert np.all(covered == 1)
    assert np.array_equal(got, want)
    ref = _expected_neighbours(w.box, w.runs)
    assert np.array_equal(zgot, ref[:, 4:6])
    assert segs.shape[0] >= g.n_segments


def test_mask_and_runs_give_same_layout(lib):
    w = configs.random_mask_problem(n=(8, 9, 10), density=0.5, seed=3)
    a = _host_grid(w.box, mask=w.extra["mask"])
    b = _host_grid(w.box, runs=w.runs)
    assert np.array_equal(a.segments(), b.segments())


def test_touching_runs_are_merged(lib):
    box = Box((2, 2, 8), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    runs = np.array([[0, 0, 0, 3], [0, 0, 3, 5], [1, 1, 2, 8]], np.int64)
    g = _host_grid(box, runs=runs)
    assert g.n_runs == 2 and g.n_active == 11
    mask = np.zeros(box.n, bool)
    mask[0, 0, 0:5] = True
    mask[1, 1, 2:8] = True
    ref = _expected_neighbours(box, runs_from_mask(mask))
    assert np.array_equal(_neighbours_from_segments(g.segments(), 11), ref)


def test_single_site_and_face_runs(lib):
    rng = np.random.default_rng(5)
    box = Box((5, 4, 7), (0.3, 0.2, 0.1), (0.0, 0.0, 0.0))
    mask = rng.random(box.n) < 0.5
    mask[0, :, :] = True       # touches the x-, y-, z- faces
    mask[-1, -1, :] = True     # and the +faces
    mask[2, 2, :] = False
    mask[2, 2, 3] = True       # an isolated 1-site run
    runs = runs_from_mask(mask)
    g = _host_grid(box, runs=runs)
    assert np.array_equal(_neighbours_from_segments(g.segments(), g.n_active), _expected_neighbours(box, runs))


def test_c1_layout(lib):
    w = configs.c1()
    g = _host_grid(w.box, runs=w.runs)
    assert (g.n_active, g.n_runs) == (40600, 2616)
    assert np.array_equal(_neighbours_from_segments(g.segments(), g.n_active), _expected_neighbours(w.box, w.runs))


def test_errors_are_reported_without_side_effects(lib):
    from paper_2603_05447_amd import GPEError
    from paper_2603_05447_amd import _lib
    box = Box((3, 3, 3), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    with pytest.raises(GPEError) as e:
        _host_grid(box, mask=np.zeros(box.n, np.uint8))
    assert e.value.status == _lib.GPE_ERR_ARG and "empty" in str(e.value)
    with pytest.raises(GPEError) as e:
        _host_grid(box, runs=np.array([[0, 0, 2, 1]], np.int64))
    assert e.value.status == _lib.GPE_ERR_ARG
    with pytest.raises(GPEError) as e:       # unsorted
        _host_grid(box, runs=np.array([[1, 0, 0, 1], [0, 0, 0, 1]], np.int64))
    assert e.value.status == _lib.GPE_ERR_ARG
    with pytest.raises(GPEError) as e:       # overlapping in one column
        _host_grid(box, runs=np.array([[0, 0, 0, 2], [0, 0, 1, 3]], np.int64))
    assert e.value.status == _lib.GPE_ERR_ARG
    with pytest.raises(GPEError) as e:       # outside the box
        _host_grid(box, runs=np.array([[0, 3, 0, 1]], np.int64))
    assert e.value.status == _lib.GPE_ERR_ARG
    geom = _lib.Geometry()
    for d in range(3):
        geom.n[d], geom.h[d], geom.x0[d] = 3, (1.0 if d else -1.0), 0.0
    h = C.c_void_p()
    m = np.ones(27, np.uint8)
    assert lib.gpe_grid_create(C.byref(geom), m.ctypes.data, -1, C.byref(h)) == _lib.GPE_ERR_ARG
    assert b"h[0]" in lib.gpe_last_error()
    # compute calls on a host-only grid: state error, nothing launched
    g = _host_grid(box, mask=np.ones(box.n, np.uint8))
    prm = _lib.Params(1.0, 1e-3, 1.0, 0, 0, 0)
    pot = _lib.Potential(0, 0, 16, 0.0, None, None)
    st = lib.gpe_imag_time(g.handle, 0, 16, C.byref(pot), C.byref(prm), 1, 16, 1 << 20, None, None, None)
    assert st == _lib.GPE_ERR_STATE
    # work sizes are host arithmetic
    b = C.c_size_t()
    assert lib.gpe_work_bytes(g.handle, 0, _lib.GPE_MODE_RT, 10, 0, C.byref(b)) == 0 and b.value >= 3 * 27 * 16
    assert lib.gpe_work_bytes(g.handle, 5, _lib.GPE_MODE_RT, 10, 0, C.byref(b)) == _lib.GPE_ERR_ARG
    # stored stage states per integrator: RKHE3 2, RK4 3, RKCK 5 (App. A)
    sizes = {}
    for mode in (_lib.GPE_MODE_RT_RKHE3, _lib.GPE_MODE_RT, _lib.GPE_MODE_RT_RKCK):
        assert lib.gpe_work_bytes(g.handle, 0, mode, 10, 0, C.byref(b)) == 0
        sizes[mode] = b.value
    assert 2 * 432 <= sizes[_lib.GPE_MODE_RT_RKHE3] < 3 * 432 <= sizes[_lib.GPE_MODE_RT] < 4 * 432
    assert 5 * 432 <= sizes[_lib.GPE_MODE_RT_RKCK] < 6 * 432 + 4096
    # imaginary time on a real state: one real per site for the temporary
    assert lib.gpe_work_bytes(g.handle, 0, _lib.GPE_MODE_ITP, 10, 0, C.byref(b)) == 0
    itp_c = b.value
    assert lib.gpe_work_bytes(g.handle, 0, _lib.GPE_MODE_ITP_REAL, 10, 0, C.byref(b)) == 0
    assert 2 * 27 * 8 <= b.value < itp_c
    assert lib.gpe_work_bytes(g.handle, 0, 6, 10, 0, C.byref(b)) == _lib.GPE_ERR_ARG
    # an unknown integrator is rejected before anything else runs
    bad = _lib.Params(1.0, 1e-3, 1.0, 0, 0, 7)
    st = lib.gpe_real_time(g.handle, 0, 16, C.byref(pot), C.byref(bad), 0.0, 1, 16, 1 << 20, None, None, None)
    assert st in (_lib.GPE_ERR_ARG, _lib.GPE_ERR_STATE)


def test_c5_scale_layout_from_analytic_runs(lib):
    """A 2048 x 2048 x 1024 box (2^32 points, int64 box indices) built from
    runs without a dense mask."""
    box = Box((2048, 2048, 1024), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    runs = []
    for i in (0, 1000, 2047):
        for j in (0, 5, 2047):
            runs.append((i, j, 0, 3))
            runs.append((i, j, 1020, 1024))
    runs = np.array(sorted(runs), np.int64)
    g = _host_grid(box, runs=runs)
    assert g.n_active == 9 * (3 + 4)
    segs = g.segments()
    assert segs[:, 1].sum() == g.n_active
    assert np.all(segs[:, 3:7] == 0)       # no lateral neighbours in this sparse set


def test_plain_c_client(lib, tmp_path):
    """The ABI is usable from C alone: a small C program (tests/c/) is built
    with gcc against include/gpe.h and libgpe.so and runs host-only calls."""
    import shutil
    import subprocess
    from paper_2603_05447_amd import _lib
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = os.path.join(ROOT, "tests", "c", "abi_host_demo.c")
    exe = str(tmp_path / "abi_host_demo")
    libdir = os.path.dirname(_lib.LIB_PATH)
    subprocess.run([gcc, "-std=c99", "-Wall", "-O1", src, "-I", os.path.join(ROOT, "include"), "-L", libdir,
                    "-lgpe", f"-Wl,-rpath,{libdir}", "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("ok ")


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
