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


# ---- 19-point HOC stencil, App. B eq. (B2) ----------------------------------

def test_19pt_constructions_agree_on_a_random_mask():
    from oracle import operator as op
    rng = np.random.default_rng(19)
    n, h = (7, 6, 8), (0.3, 0.45, 0.25)
    mask = rng.uniform(size=n) < 0.55
    lin = np.flatnonzero(mask.ravel())
    A = op.kinetic_kron_19(n, h, lin).toarray()
    B = op.kinetic_direct_19(n, h, lin).toarray()
    assert np.max(np.abs(A - B)) <= 1e-12 * np.max(np.abs(A))
    assert np.max(np.abs(A - A.T)) == 0.0                      # restriction keeps the symmetry


def test_19pt_full_box_spectrum_closed_form():
    """On the full box the Dirichlet sine modes diagonalise every Kronecker
    factor, so the eigenvalues of eq. (B2) are sum_d mu_d + (1/12) sum_{a<b}
    (h_a^2 + h_b^2) mu_a mu_b with mu_d = -(4/h_d^2) sin^2(k_d pi / (2(n_d + 1)))."""
    from oracle import operator as op
    n, h = (5, 4, 6), (0.5, 0.35, 0.6)
    lin = np.arange(n[0] * n[1] * n[2])
    T = op.kinetic_kron_19(n, h, lin).toarray()
    mu = [-(4.0 / h[d] ** 2) * np.sin(np.arange(1, n[d] + 1) * np.pi / (2 * (n[d] + 1))) ** 2 for d in range(3)]
    a, b, c = np.meshgrid(mu[0], mu[1], mu[2], indexing="ij")
    h2 = [v * v for v in h]
    lam = a + b + c + ((h2[0] + h2[1]) * a * b + (h2[0] + h2[2]) * a * c + (h2[1] + h2[2]) * b * c) / 12.0
    want = np.sort((-0.5 * lam).ravel())
    got = np.linalg.eigvalsh(T)
    assert np.max(np.abs(np.sort(got) - want)) <= 1e-11 * np.max(np.abs(want))


def test_19pt_isotropic_weights_are_the_classical_stencil():
    """For equal spacings eq. (B2) is the classical 19-point Laplacian
    (1/(6 h^2)) [-24 at the centre, 2 at the faces, 1 at the edges]."""
    from oracle import operator as op
    h = 0.37
    w = op.stencil_19_weights((h, h, h))
    assert len(w) == 19
    for off, v in w.items():
        nz = sum(1 for x in off if x != 0)
        want = {0: -24.0, 1: 2.0, 2: 1.0}[nz] / (6 * h * h)
        assert abs(v - want) <= 1e-13 * abs(want)


@pytest.mark.parametrize("aniso", [False, True])
def test_19pt_truncation_error_is_fourth_order_beyond_the_hoc_term(aniso):
    """Taylor expansion: the 19-point operator equals Lap u + (1/12)[sum_d h_d^2
    d_d^4 u + sum_{a<b} (h_a^2 + h_b^2) d_a^2 d_b^2 u] + O(h^4).  Checked on a
    Gaussian (closed-form derivatives) at interior points: halving h cuts the
    remainder by ~16, which fails for a wrong 1/12 or a wrong sign."""
    from oracle import operator as op

    def remainder(hs):
        L = 6.0
        n = tuple(int(round(2 * L / hd)) for hd in hs)
        ax = [-L + (np.arange(n[d]) + 0.5) * hs[d] for d in range(3)]
        x, y, z = np.meshgrid(*ax, indexing="ij")
        G = np.exp(-(x * x + y * y + z * z) / 2)
        lin = np.arange(G.size)
        Lu = (-2.0 * op.kinetic_direct_19(n, hs, lin) @ G.ravel()).reshape(n)
        c = [x, y, z]
        d2 = [(v * v - 1) for v in c]
        d4 = [(v ** 4 - 6 * v * v + 3) for v in c]
        lap = (d2[0] + d2[1] + d2[2]) * G
        hoc = sum(hs[d] ** 2 * d4[d] for d in range(3))
        for a in range(3):
            for b in range(a + 1, 3):
                hoc = hoc + (hs[a] ** 2 + hs[b] ** 2) * d2[a] * d2[b]
        ref = lap + hoc * G / 12.0
        inner = (np.abs(x) < 2.5) & (np.abs(y) < 2.5) & (np.abs(z) < 2.5)
        return np.max(np.abs(Lu - ref)[inner])

    base = (0.4, 0.5, 0.3) if aniso else (0.4, 0.4, 0.4)
    e1 = remainder(base)
    e2 = remainder(tuple(v / 2 for v in base))
    assert 12.0 < e1 / e2 < 20.0


# ---- cubic 27-point stencil (equal spacings) ---------------------------------

def test_27pt_constructions_agree_and_spectrum_closed_form():
    """Kronecker construction vs direct assembly on a random mask; on the full
    box the sine modes give eigenvalues (1/(30 h^2)) [-128 + 28 sum c_d +
    12 sum_{a<b} c_a c_b + 8 c_x c_y c_z], c_d = cos(k_d pi / (n_d + 1))."""
    from oracle import operator as op
    rng = np.random.default_rng(27)
    n, h = (6, 5, 7), (0.35, 0.35, 0.35)
    lin = np.flatnonzero(rng.uniform(size=n).ravel() < 0.6)
    A = op.kinetic_kron_27(n, h, lin).toarray()
    B = op.kinetic_direct_27(n, h, lin).toarray()
    assert np.max(np.abs(A - B)) <= 1e-12 * np.max(np.abs(A))
    assert np.max(np.abs(A - A.T)) == 0.0
    full = np.arange(n[0] * n[1] * n[2])
    T = op.kinetic_direct_27(n, h, full).toarray()
    c = [np.cos(np.arange(1, n[d] + 1) * np.pi / (n[d] + 1)) for d in range(3)]
    x, y, z = np.meshgrid(c[0], c[1], c[2], indexing="ij")
    lam = (-128 + 28 * (x + y + z) + 12 * (x * y + x * z + y * z) + 8 * x * y * z) / (30 * h[0] ** 2)
    want = np.sort((-0.5 * lam).ravel())
    assert np.max(np.abs(np.linalg.eigvalsh(T) - want)) <= 1e-11 * np.max(np.abs(want))
    with pytest.raises(ValueError):
        op.kinetic_kron_27(n, (0.3, 0.35, 0.35), lin)


def test_27pt_truncation_error_is_fourth_order_beyond_the_hoc_term():
    """Lap_27 u = Lap u + (h^2/12) Lap^2 u + O(h^4) on a Gaussian (closed-form
    derivatives): halving h cuts the remainder by ~16."""
    from oracle import operator as op

    def remainder(hh):
        L = 6.0
        n = (int(round(2 * L / hh)),) * 3
        ax = -L + (np.arange(n[0]) + 0.5) * hh
        x, y, z = np.meshgrid(ax, ax, ax, indexing="ij")
        r2 = x * x + y * y + z * z
        G = np.exp(-r2 / 2)
        Lu = (-2.0 * op.kinetic_direct_27(n, (hh, hh, hh), np.arange(G.size)) @ G.ravel()).reshape(n)
        ref = (r2 - 3) * G + (hh * hh / 12) * (r2 * r2 - 10 * r2 + 15) * G
        inner = (np.abs(x) < 2.5) & (np.abs(y) < 2.5) & (np.abs(z) < 2.5)
        return np.max(np.abs(Lu - ref)[inner])

    e1, e2 = remainder(0.4), remainder(0.2)
    assert 12.0 < e1 / e2 < 20.0
