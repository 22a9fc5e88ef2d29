"""Staged ramps with re-post-selection (oracle; test infrastructure).

Sec. V runs the detuning ramp as a sequence of stages between precomputed
potentials V_0, V_1, ..., V_S on the full Cartesian grid.  Within stage i
the potential is interpolated linearly in time between V_i and V_{i+1}.
At the end of every stage the grid post-selection of Sec. II.A (keep the
points below a cutoff, drop the rest) is repeated with the cutoff
5 max(mu_i, mu_{i+1}), mu_i being the chemical potential of the ground state
in V_i, and the wavefunction is carried over from the old grid to the new
one.

Readings (the paper gives no formulas for these):
* the region kept for stage i is where min(V_i, V_{i+1}) is below the
  cutoff, so that every potential met during the stage is covered (the
  interpolated V(t) is never below that minimum);
* carrying psi over copies the value of every point kept by both grids,
  sets the newly added points to zero and drops the removed ones (no
  renormalisation: the stage's own evolution is unitary up to the dropped
  tail);
* time within stage i runs from t_i to t_{i+1}; before t_i the stage
  potential is V_i, after t_{i+1} it is V_{i+1}.

Everything here is defined on box linear indices, so it needs no layout
structure beyond the sorted list of active box indices of each grid.
"""
from __future__ import annotations

import numpy as np


class LerpPotential:
    """V(t) = (1 - lam) V_a + lam V_b, lam = clamp((t - t_a)/(t_b - t_a), 0, 1)."""

    def __init__(self, Va: np.ndarray, Vb: np.ndarray, ta: float, tb: float):
        self.Va = np.asarray(Va, float)
        self.Vb = np.asarray(Vb, float)
        self.ta = float(ta)
        self.tb = float(tb)

    def lam(self, t: float) -> float:
        return min(max((t - self.ta) / (self.tb - self.ta), 0.0), 1.0)

    def __call__(self, t: float) -> np.ndarray:
        lam = self.lam(t)
        return (1.0 - lam) * self.Va + lam * self.Vb


def post_select(Va_box: np.ndarray, Vb_box, cutoff: float) -> np.ndarray:
    """Boolean box mask of the points kept for a stage between Va and Vb
    (Vb may be None for a single potential)."""
    v = np.asarray(Va_box, float)
    if Vb_box is not None:
        v = np.minimum(v, np.asarray(Vb_box, float))
    return v < cutoff


def stage_cutoff(mu_i: float, mu_next: float) -> float:
    return 5.0 * max(mu_i, mu_next)


def remap(psi_src: np.ndarray, lin_src: np.ndarray, lin_dst: np.ndarray) -> np.ndarray:
    """Carry psi from the grid with sorted active box indices lin_src to the
    grid with lin_dst: common points keep their value, new points are zero."""
    lin_src = np.asarray(lin_src, np.int64)
    lin_dst = np.asarray(lin_dst, np.int64)
    out = np.zeros(lin_dst.size, dtype=np.asarray(psi_src).dtype)
    pos = np.searchsorted(lin_src, lin_dst)
    pos_c = np.minimum(pos, max(lin_src.size - 1, 0))
    hit = (lin_src.size > 0) & (lin_src[pos_c] == lin_dst)
    out[hit] = np.asarray(psi_src)[pos_c[hit]]
    return out
