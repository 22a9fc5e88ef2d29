"""Pins for the oracle's reduced kinetic operator T~ (Sec. II.A, App. B eq. (B1))."""
import numpy as np
import pytest

from oracle import operator as op
from oracle import dense
from workloads import configs, Box, runs_from_mask, site_linear_index, site_ijk


def brute_force_T_apply(box, mask, psi_box):
    """Explicit per-site loop: -1/2 sum_d (psi(+e_d) + psi(-e_d) - 2 psi)/h_d^2,
    psi = 0 outside the mask and outside the box."""
    n0, n1, n2 = box.n
    out = np.zeros_like(psi_box)
    for i in range(n0):
        for j in range(n1):
            for k in range(n2):
                if not mask[i, j, k]:
                    continue
                c = psi_box[i, j, k]
                acc = 0.0
                for d, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
                    s = 0.0
                    for sg in (1, -1):
                        a, b, e = i + sg * di, j + sg * dj, k + sg * dk
                        if 0 <= a < n0 and 0 <= b < n1 and 0 <= e < n2 and mask[a, b, e]:
                            s = s + psi_box[a, b, e]
                    acc = acc + (s - 2.0 * c) / box.h[d] ** 2
                out[i, j, k] = -0.5 * acc
    return out


@pytest.mark.parametrize("seed,density", [(1, 0.3), (2, 0.6), (3, 0.95)])
def test_T_matches_explicit_loop(seed, density):
    w = configs.random_mask_problem(n=(7, 6, 9), density=density, seed=seed)
    mask = w.extra["mask"]
    lin = site_linear_index(w.box, w.runs)
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(lin.size) + 1j * rng.standard_normal(lin.size)
    box_psi = np.zeros(w.box.n, complex)
    box_psi.ravel()[lin] = psi
    ref = brute_force_T_apply(w.box, mask, box_psi).ravel()[lin]
    for T in (op.kinetic_direct(w.box.n, w.box.h, lin), op.kinetic_kron(w.box.n, w.box.h, lin)):
        got = op.apply(T, psi)
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_two_constructions_agree_on_shell():
    w = configs.small_shell(n=24)
    lin = site_linear_index(w.box, w.runs)
    A = op.kinetic_direct(w.box.n, w.box.h, lin)
    B = op.kinetic_kron(w.box.n, w.box.h, lin)
    d = (A - B).tocsr()
    assert abs(d).max() <= 1e-14 * abs(A).max()
    assert A.nnz == B.nnz
    # symmetric, and every row has at most 7 entries (7-point stencil)
    assert abs(A - A.T).max() == 0.0
    assert np.max(np.diff(A.indptr)) <= 7


def test_full_box_spectrum_closed_form():
    """Full box, Dirichlet: eigenvalues are 1/2 sum_d (4/h_d^2) sin^2(k_d pi / (2 (n_d + 1)))."""
    box = Box((4, 5, 6), (0.5, 0.45, 0.4), (0.0, 0.0, 0.0))
    runs = runs_from_mask(np.ones(box.n, bool))
    lin = site_linear_index(box, runs)
    T = op.kinetic_direct(box.n, box.h, lin).toarray()
    ev = np.sort(np.linalg.eigvalsh(T))
    ks = [np.arange(1, box.n[d] + 1) for d in range(3)]
    lam = [(4.0 / box.h[d] ** 2) * np.sin(ks[d] * np.pi / (2 * (box.n[d] + 1))) ** 2 for d in range(3)]
    closed = 0.5 * (lam[0][:, None, None] + lam[1][None, :, None] + lam[2][None, None, :])
    assert np.allclose(ev, np.sort(closed.ravel()), rtol=0, atol=1e-12 * closed.max())


def test_dense_kinetic_matches_masked_on_full_box():
    box = Box.centred((5, 4, 6), (1.0, 1.2, 0.9))
    runs = runs_from_mask(np.ones(box.n, bool))
    lin = site_linear_index(box, runs)
    T = op.kinetic_direct(box.n, box.h, lin).toarray()
    D = dense.dense_kinetic(box.n, box.h)
    assert np.max(np.abs(T - D)) <= 1e-14 * np.max(np.abs(D))


def test_c1_geometry_counts():
    """C1 geometry: 64^3 cell-centred box on [-8,8)^3 with V = 20 (r-5)^2 < 20."""
    w = configs.c1()
    assert w.n_active == 40600
    assert w.runs.shape[0] == 2616
    i, j, k = site_ijk(w.runs)
    lin = (i * 64 + j) * 64 + k
    assert np.all(np.diff(lin) > 0)
