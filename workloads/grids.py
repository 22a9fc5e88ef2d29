"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only builds problem data: box geometry, active-site runs, the
fields that define a potential on the active sites, and seeded initial
states.  It contains none of the solver's arithmetic (no Laplacian, no time
stepping, no observables); both the CPU oracle and the HIP path receive what
is built here and nothing else.

Geometry convention (cell-centred, z fastest):
    site (i, j, k) sits at x0 + (i, j, k) * h, box linear index
    (i * n1 + j) * n2 + k.  A box of half-widths L_d with n_d points has
    h_d = 2 L_d / n_d and x0_d = -L_d + h_d / 2.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Tuple

import numpy as np


@dataclass(frozen=True)
class Box:
    n: Tuple[int, int, int]
    h: Tuple[float, float, float]
    x0: Tuple[float, float, float]

    @staticmethod
    def centred(n, half_width) -> "Box":
        n = tuple(int(v) for v in (n if np.ndim(n) else (n, n, n)))
        L = tuple(float(v) for v in (half_width if np.ndim(half_width) else (half_width,) * 3))
        h = tuple(2.0 * L[d] / n[d] for d in range(3))
        x0 = tuple(-L[d] + 0.5 * h[d] for d in range(3))
        return Box(n, h, x0)

    def axis(self, d: int) -> np.ndarray:
        return self.x0[d] + self.h[d] * np.arange(self.n[d], dtype=np.float64)

    @property
    def dV(self) -> float:
        return self.h[0] * self.h[1] * self.h[2]

    @property
    def size(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]


def runs_from_predicate(box: Box, active: Callable[[np.ndarray, np.ndarray, np.ndarray], np.ndarray]) -> np.ndarray:
    """Scan the box one x-plane at a time and return the z-runs of the active set.

    `active(x, y, z)` gets broadcastable coordinate arrays of one plane and
    returns a boolean (n1, n2) array.  Result: int64 array (nruns, 4) of
    (i, j, k0, k1), k1 exclusive, sorted by (i, j, k0).
    """
    xs, ys, zs = box.axis(0), box.axis(1), box.axis(2)
    Y = ys[:, None]
    Z = zs[None, :]
    out = []
    for i in range(box.n[0]):
        m = np.asarray(active(xs[i], Y, Z), dtype=bool)
        m = np.broadcast_to(m, (box.n[1], box.n[2]))
        out.append(_plane_runs(i, m))
    if not out:
        return np.zeros((0, 4), np.int64)
    return np.concatenate(out, axis=0)


def _plane_runs(i: int, m: np.ndarray) -> np.ndarray:
    n1, n2 = m.shape
    p = np.zeros((n1, n2 + 2), np.int8)
    p[:, 1:-1] = m
    d = np.diff(p, axis=1)
    js, k0 = np.nonzero(d == 1)
    je, k1 = np.nonzero(d == -1)
    assert np.array_equal(js, je)
    r = np.empty((js.size, 4), np.int64)
    r[:, 0] = i
    r[:, 1] = js
    r[:, 2] = k0
    r[:, 3] = k1
    return r


def runs_from_mask(mask: np.ndarray) -> np.ndarray:
    mask = np.asarray(mask, dtype=bool)
    out = [_plane_runs(i, mask[i]) for i in range(mask.shape[0])]
    return np.concatenate(out, axis=0) if out else np.zeros((0, 4), np.int64)


def mask_from_runs(box: Box, runs: np.ndarray) -> np.ndarray:
    m = np.zeros(box.n, dtype=bool)
    for i, j, k0, k1 in np.asarray(runs):
        m[i, j, k0:k1] = True
    return m


def site_ijk(runs: np.ndarray):
    """Per-site (i, j, k) in compact order (C order restricted to the active set)."""
    runs = np.asarray(runs, dtype=np.int64)
    lens = runs[:, 3] - runs[:, 2]
    n = int(lens.sum())
    rid = np.repeat(np.arange(runs.shape[0]), lens)
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]]) if runs.shape[0] else np.zeros(0, np.int64)
    k = runs[rid, 2] + (np.arange(n) - starts[rid])
    return runs[rid, 0], runs[rid, 1], k


def site_coords(box: Box, runs: np.ndarray):
    i, j, k = site_ijk(runs)
    return (box.x0[0] + box.h[0] * i, box.x0[1] + box.h[1] * j, box.x0[2] + box.h[2] * k)


def site_linear_index(box: Box, runs: np.ndarray) -> np.ndarray:
    i, j, k = site_ijk(runs)
    return (i * box.n[1] + j) * box.n[2] + k


def complex_noise(rng: np.random.Generator, n: int, amplitude: float) -> np.ndarray:
    re = rng.uniform(-1.0, 1.0, size=n)
    im = rng.uniform(-1.0, 1.0, size=n)
    return amplitude * (re + 1j * im)


def normalise_input(psi: np.ndarray, dV: float, norm: float = 1.0) -> np.ndarray:
    """Scale an initial state so that dV * sum |psi|^2 = norm (the input's
    normalisation condition, eq. (3)); used only to prepare inputs."""
    s = float(np.sum(psi.real ** 2 + psi.imag ** 2)) * dV
    return psi * np.sqrt(norm / s)
