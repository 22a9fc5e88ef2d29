"""Pins for the oracle's staged-ramp pieces (Sec. V): the interpolated
stage potential, the post-selection mask and the carry-over of psi between
grids, against closed forms and brute force on tiny boxes."""
import numpy as np

from oracle import restage
from oracle import realtime as rt
from oracle import operator as op
from oracle.potential import StaticPotential
from workloads import Box, runs_from_mask, site_linear_index


def test_lerp_potential_closed_forms():
    rng = np.random.default_rng(0)
    Va, Vb = rng.uniform(0, 5, 50), rng.uniform(0, 5, 50)
    p = restage.LerpPotential(Va, Vb, 0.3, 0.7)
    assert np.array_equal(p(0.3), Va) and np.array_equal(p(0.7), Vb)
    assert np.array_equal(p(-1.0), Va) and np.array_equal(p(5.0), Vb)      # held outside the stage
    assert np.allclose(p(0.5), 0.5 * (Va + Vb), rtol=0, atol=1e-15)
    # affine in t inside the stage: vanishing second difference
    t = 0.41
    assert np.max(np.abs(p(t - 0.05) - 2 * p(t) + p(t + 0.05))) < 1e-14


def test_post_select_matches_brute_force():
    rng = np.random.default_rng(1)
    n = (5, 4, 6)
    Va, Vb = rng.uniform(0, 10, n), rng.uniform(0, 10, n)
    cut = 4.0
    m = restage.post_select(Va, Vb, cut)
    for i in range(n[0]):
        for j in range(n[1]):
            for k in range(n[2]):
                keep = (Va[i, j, k] < cut) or (Vb[i, j, k] < cut)
                assert m[i, j, k] == keep
    assert np.array_equal(restage.post_select(Va, None, cut), Va < cut)
    assert np.all(restage.post_select(Va, Vb, cut + 1.0) >= m)        # a larger cutoff keeps a superset
    assert restage.stage_cutoff(2.0, 3.5) == 17.5


def _lin(box, mask):
    return site_linear_index(box, runs_from_mask(mask))


def test_remap_against_a_lookup_table():
    rng = np.random.default_rng(2)
    box = Box.centred((6, 5, 7), 3.0)
    ma = rng.uniform(size=box.n) < 0.5
    mb = rng.uniform(size=box.n) < 0.5
    la, lb = _lin(box, ma), _lin(box, mb)
    psi = rng.standard_normal(la.size) + 1j * rng.standard_normal(la.size)
    out = restage.remap(psi, la, lb)
    table = {int(x): psi[q] for q, x in enumerate(la)}
    for q, x in enumerate(lb):
        assert out[q] == table.get(int(x), 0.0)
    # the mass carried over is exactly the mass on the common points
    common = np.isin(la, lb)
    assert np.sum(np.abs(out) ** 2) == np.sum(np.abs(psi[common]) ** 2)


def test_remap_identity_and_round_trip_through_a_superset():
    rng = np.random.default_rng(3)
    box = Box.centred((7, 6, 5), 3.0)
    m = rng.uniform(size=box.n) < 0.4
    sup = m | (rng.uniform(size=box.n) < 0.3)
    l, ls = _lin(box, m), _lin(box, sup)
    psi = rng.standard_normal(l.size) + 1j * rng.standard_normal(l.size)
    assert np.array_equal(restage.remap(psi, l, l), psi)
    assert np.array_equal(restage.remap(restage.remap(psi, l, ls), ls, l), psi)
    empty = restage.remap(psi, l, np.zeros(0, np.int64))
    assert empty.size == 0


def test_a_stage_with_equal_end_potentials_is_the_static_run():
    rng = np.random.default_rng(4)
    box = Box.centred(6, 3.0)
    mask = rng.uniform(size=box.n) < 0.6
    lin = _lin(box, mask)
    T = op.kinetic_direct(box.n, box.h, lin)
    V = rng.uniform(0, 3, lin.size)
    psi = (rng.standard_normal(lin.size) + 1j * rng.standard_normal(lin.size)) * 0.1
    a = rt.real_time(T, psi, restage.LerpPotential(V, V, 0.0, 0.1), 2.0, 1e-3, 0.0, 20)
    b = rt.real_time(T, psi, StaticPotential(V), 2.0, 1e-3, 0.0, 20)
    # (1 - lam) V + lam V equals V up to one rounding per evaluation
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))
