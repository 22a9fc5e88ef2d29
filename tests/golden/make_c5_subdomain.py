"""Write the FP64 oracle's reference for the C5 precision study on a
downscaled subdomain (test infrastructure; calls only `oracle/` and the
seeded input generators in `workloads/`).

The instance is `workloads.configs.c5_subdomain(scale)`: the large thin
shell shrunk by `scale` per axis at the same spacing, so the shell keeps its
thickness in grid units (mean z-run 10.7 sites, as in the full shell).  The
oracle integrates eq. (8) with classic RK4 in k-form for the full 20,000
steps of dt = 5e-5 and records
  * norm, energy and chemical potential every `obs_every` steps, and
  * the state at a seeded sample of sites after 20, 200, 2000 and 20,000
    steps,
in `c5_subdomain_s<scale>.npz` beside this script.

Usage: OMP_NUM_THREADS=1 python tests/golden/make_c5_subdomain.py [scale]
(scale 8: 931,864 sites, about 80 minutes on one core; scale 4: 3,732,680
sites, about 5 hours).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import operator as op  # noqa: E402
from oracle import realtime as rt  # noqa: E402
from oracle.observables import energy_mu  # noqa: E402
from oracle.potential import RFRamp  # noqa: E402
from workloads import configs, site_linear_index  # noqa: E402

SAMPLE_STEPS = (20, 200, 2000, 20000)
N_SAMPLES = 8192


def sample_sites(n_active: int, seed: int = 55) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_active, size=min(N_SAMPLES, n_active), replace=False)).astype(np.int64)


def main(scale: int = 8, obs_every: int = 1000) -> str:
    w = configs.c5_subdomain(scale)
    lin = site_linear_index(w.box, w.runs)
    T = op.kinetic_direct(w.box.n, w.box.h, lin)
    ramp = RFRamp(w.field, w.omega, w.knot_t, w.knot_delta)
    idx = sample_sites(w.n_active)
    obs_steps, obs_vals, samples = [], [], {}
    y = np.array(w.psi0, dtype=np.complex128, copy=True)
    t0 = time.time()
    for n in range(w.steps + 1):
        if n % obs_every == 0:
            obs_steps.append(n)
            obs_vals.append(energy_mu(T, y, ramp(n * w.dt), w.g, w.box.dV))
        if n in SAMPLE_STEPS:
            samples[n] = y[idx].copy()
        if n == w.steps:
            break
        y = rt.rk4_step(T, y, n * w.dt, w.dt, ramp, w.g)
        if (n + 1) % 500 == 0:
            el = time.time() - t0
            print(f"step {n + 1}/{w.steps}  {el:.0f} s  ({w.n_active * (n + 1) / el:.3e} site updates/s)", flush=True)
    out = os.path.join(HERE, f"c5_subdomain_s{scale}.npz")
    np.savez_compressed(out, scale=scale, n_active=w.n_active, steps=w.steps, dt=w.dt, g=w.g,
                        sample_index=idx, sample_steps=np.array(SAMPLE_STEPS, dtype=np.int64),
                        samples=np.stack([samples[s] for s in SAMPLE_STEPS]),
                        obs_steps=np.array(obs_steps, dtype=np.int64), obs=np.array(obs_vals, dtype=np.float64))
    print(f"wrote {out} ({time.time() - t0:.0f} s)", flush=True)
    return out


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 8)
