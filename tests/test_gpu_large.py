"""Maximum-size parity: a full 704^3 box (348,913,664 active sites), whose
complex128 arrays (5.6 GB each) are past 4 GiB, so every pass runs the
kernels compiled with 64-bit addressing.

The inputs are closed-form functions of the coordinates, evaluated on the
device for the whole box and on the host for each oracle patch (no 5.6 GB
host arrays).  As in the RF bubble full-size test, the oracle runs on the
active sites of a 13^3 patch around each sampled site (one RK4 step moves
information 4 sites, one imaginary-time step 2); the imaginary-time result
is compared up to its global renormalisation factor."""
import numpy as np
import pytest

from oracle import operator as op, itp, realtime as rt
from oracle.potential import StaticPotential
from gpu_cases import parity_err
from workloads import Box

pytestmark = pytest.mark.gpu
N = 704
R_PATCH = 6


@pytest.fixture(scope="module")
def big():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_05447_amd import Grid
    box = Box.centred(N, 17.6)
    ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    runs = np.stack([ii.ravel(), jj.ravel(), np.zeros(N * N, np.int64), np.full(N * N, N)], axis=1)
    print(f"large box {N}^3: building the layout", flush=True)
    g = Grid.from_box(box, runs=runs.astype(np.int64), device=0)
    assert g.n_active == N ** 3
    return box, g


def _fields(x, y, z, lib):
    """psi and V as functions of the coordinates (numpy or torch)."""
    r2 = x * x + y * y + z * z
    amp = (1.0 + 0.3 * lib.sin(2.0 * x) * lib.cos(3.0 * y)) * lib.exp(-r2 / 50.0)
    ph = 0.7 * x - 0.4 * z + 0.2 * y
    V = 0.5 * (x * x + 2.0 * y * y + 3.0 * z * z)
    return amp * lib.cos(ph), amp * lib.sin(ph), V


def _device_inputs(box):
    import torch
    ax = [torch.tensor(box.axis(d), dtype=torch.float64, device="cuda:0") for d in range(3)]
    x, y, z = ax[0][:, None, None], ax[1][None, :, None], ax[2][None, None, :]
    re, im, V = _fields(x, y, z, torch)
    psi = torch.complex(re, im).reshape(-1).contiguous()
    del re, im
    return psi, V.reshape(-1).contiguous()


def _patch(box, s):
    n = box.n
    ci, cj, ck = s // (n[1] * n[2]), (s // n[2]) % n[1], s % n[2]
    rng_ = [np.arange(max(c - R_PATCH, 0), min(c + R_PATCH, n[d] - 1) + 1) for d, c in enumerate((ci, cj, ck))]
    I, J, K = np.meshgrid(*rng_, indexing="ij")
    lin = ((I * n[1] + J) * n[2] + K).ravel()
    x = box.x0[0] + box.h[0] * I.ravel()
    y = box.x0[1] + box.h[1] * J.ravel()
    z = box.x0[2] + box.h[2] * K.ravel()
    re, im, V = _fields(x, y, z, np)
    T = op.kinetic_direct(n, box.h, lin)
    return T, re + 1j * im, V, int(np.searchsorted(lin, s))


def _samples(seed):
    rng = np.random.default_rng(seed)
    n = N ** 3
    s = list(rng.integers(0, n, 30)) + [0, n - 1, N - 1, N * N * (N // 2) + N * (N // 2) + N // 2,
                                        n - N * N + 5]
    return sorted(set(int(v) for v in s))


def test_large_box_rk4_step_with_64bit_addressing(big):
    import torch
    from paper_2603_05447_amd import Potential
    box, g = big
    psi, V = _device_inputs(box)
    dt, gg = 5e-4, 50.0
    print("large box: one RK4 step", flush=True)
    g.real_time(psi, Potential.static(V), gg, dt, 1, observe=False)
    samples = _samples(0)
    got = psi[torch.tensor(samples, device="cuda:0")].cpu().numpy()
    ref = []
    for s in samples:
        T, p0, Vp, c = _patch(box, s)
        ref.append(rt.rk4_step(T, p0, 0.0, dt, StaticPotential(Vp), gg)[c])
    ref = np.array(ref)
    err = parity_err(got, ref)
    print(f"  sampled parity error = {err:.3e}", flush=True)
    assert err <= 1e-10


def test_large_box_imag_time_step_with_64bit_addressing(big):
    import torch
    from paper_2603_05447_amd import Potential
    box, g = big
    psi, V = _device_inputs(box)
    dt, gg = 1e-3, 50.0
    print("large box: one imaginary-time step", flush=True)
    obs = g.imag_time(psi, Potential.static(V), gg, dt, 1)
    assert abs(obs["norm"] - 1.0) < 1e-12
    samples = _samples(1)
    got = psi[torch.tensor(samples, device="cuda:0")].cpu().numpy()
    ref = []
    for s in samples:
        T, p0, Vp, c = _patch(box, s)
        y, nrm = itp.itp_step(T, p0, itp.propagator(Vp, dt), gg, dt, box.dV)
        ref.append(y[c] * np.sqrt(nrm))
    ref = np.array(ref)
    scale = np.real(np.vdot(ref, got)) / np.real(np.vdot(ref, ref))
    assert scale > 0
    err = parity_err(got, scale * ref)
    print(f"  sampled parity error (up to the global scale) = {err:.3e}", flush=True)
    assert err <= 1e-10
