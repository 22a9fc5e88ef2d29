"""Helpers shared by the GPU parity tests: put a seeded workload on the
device through the binding, and run the oracle on the same inputs."""
from __future__ import annotations

import numpy as np

from oracle import operator as op
from oracle.potential import StaticPotential, RFRamp, ShellRamp
from workloads import site_linear_index


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# An aggregate relative L2 over many sites can hide a single bad site, so the
# parity measure also bounds every element: max|a - b| <= ELEMENT_FACTOR *
# tol * max|b| whenever parity_err(a, b) <= tol.
ELEMENT_FACTOR = 10.0


def max_rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def parity_err(a, b) -> float:
    """The larger of the relative L2 error and the element-wise error
    max|a - b| / max|b| scaled down by ELEMENT_FACTOR."""
    return max(rel_l2(a, b), max_rel(a, b) / ELEMENT_FACTOR)


def ramp_of(w):
    """The batch ramp tuple (omega, knot_t, knot_values, kind) of a workload."""
    from paper_2603_05447_amd import GPE_POT_RF_RAMP, GPE_POT_SHELL_RAMP
    return (w.omega, w.knot_t, w.knot_delta, GPE_POT_SHELL_RAMP if w.kind == "shell" else GPE_POT_RF_RAMP)


def oracle_ramp(w, field=None, knot_delta=None):
    """The oracle's potential of a ramped workload (optionally on a subset of
    its field and with other knot values)."""
    f = w.field if field is None else field
    kd = w.knot_delta if knot_delta is None else knot_delta
    if w.kind == "shell":
        return ShellRamp(f, w.omega, w.knot_t, kd)
    return RFRamp(f, w.omega, w.knot_t, kd)


def device_ramp(w, field):
    """The binding's potential of a ramped workload on a device field."""
    from paper_2603_05447_amd import Potential
    if w.kind == "shell":
        return Potential.shell(field, w.omega, w.knot_t, w.knot_delta)
    return Potential.rf(field, w.omega, w.knot_t, w.knot_delta)


class Case:
    """A workload on the GPU (binding objects) and on the CPU (oracle objects)."""

    def __init__(self, w, dtype="c128", config=None):
        import torch
        from paper_2603_05447_amd import Grid, Potential

        self.w = w
        self.dev = torch.device("cuda:0")
        self.cdt = torch.complex128 if dtype == "c128" else torch.complex64
        self.rdt = torch.float64 if dtype == "c128" else torch.float32
        self.grid = Grid.from_box(w.box, runs=w.runs, device=0)
        if config is not None:
            self.grid.set_config(config)
        self.field = torch.tensor(w.field, dtype=self.rdt, device=self.dev)
        if w.kind in ("rf", "shell"):
            self.pot = device_ramp(w, self.field)
            self.opot = oracle_ramp(w)
        else:
            self.pot = Potential.static(self.field)
            self.opot = StaticPotential(w.field)
        self._T = None

    @property
    def T(self):
        if self._T is None:
            lin = site_linear_index(self.w.box, self.w.runs)
            self._T = op.kinetic_direct(self.w.box.n, self.w.box.h, lin)
        return self._T

    def psi(self, arr=None):
        import torch
        a = self.w.psi0 if arr is None else arr
        return torch.tensor(np.asarray(a), dtype=self.cdt, device=self.dev)
