"""Reduced kinetic operator T~ on the active set (oracle; test infrastructure).

Sec. II.A builds the Laplacian of the full Cartesian grid from outer
(Kronecker) products of identity matrices and the 1D second-order central
difference matrices, then removes every row and column of a grid point
outside the region of interest; T~ carries the prefactor -hbar^2/2m.  App. B
eq. (B1) gives the anisotropic weights: delta_d^2 = [1, -2, 1] / d_d^2.
Removing the rows/columns is the same as imposing psi = 0 off the active set
(Dirichlet), and the box edge is Dirichlet as well.

Two independent constructions are provided and must agree:
* `kinetic_kron`   - the paper's literal construction (Kronecker sum over the
                     whole box, then row/column removal); memory ~ box size;
* `kinetic_direct` - direct CSR assembly from the sorted active box indices
                     (searchsorted on the +-1, +-n2, +-n1*n2 shifts);
                     memory ~ number of active sites.

The 19-point higher-order compact (HOC) stencil of App. B eq. (B2) adds to
the Kronecker sum the mixed terms (1/12)(d_a^2 + d_b^2) delta_a^2 (x) delta_b^2
for each pair of axes (a, b); the same two constructions are provided for it
(`kinetic_kron_19`, `kinetic_direct_19`), and for the cubic 27-point stencil
used in Sec. II.B / III (weights not printed; taken here for equal spacings
as (1/(30 h^2)) [-128, 14, 3, 1] at the centre, faces, edges and corners, a
stencil whose leading error is the same isotropic (h^2/12) Lap^2 as eq.
(B2)'s) (`kinetic_kron_27`, `kinetic_direct_27`).

Sites are ordered by box linear index (i*n1 + j)*n2 + k (z fastest).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def second_difference_1d(n: int, h: float) -> sp.csr_matrix:
    """delta^2 = [1, -2, 1] / h^2 with Dirichlet ends (App. B)."""
    main = np.full(n, -2.0 / (h * h))
    off = np.full(n - 1, 1.0 / (h * h))
    return sp.diags([off, main, off], [-1, 0, 1], shape=(n, n), format="csr")


def laplacian_kron(n, h) -> sp.csr_matrix:
    """Full-box 7-point Laplacian as the Kronecker sum of eq. (B1)."""
    Dx, Dy, Dz = (second_difference_1d(n[d], h[d]) for d in range(3))
    Ix, Iy, Iz = (sp.identity(n[d], format="csr") for d in range(3))
    L = sp.kron(sp.kron(Dx, Iy), Iz) + sp.kron(sp.kron(Ix, Dy), Iz) + sp.kron(sp.kron(Ix, Iy), Dz)
    return L.tocsr()


def kinetic_kron(n, h, lin: np.ndarray) -> sp.csr_matrix:
    """T~ = -1/2 * (Laplacian with the rows and columns outside the ROI removed)."""
    L = laplacian_kron(n, h)
    lin = np.asarray(lin, dtype=np.int64)
    return (-0.5 * L[lin][:, lin]).tocsr()


def kinetic_direct(n, h, lin: np.ndarray) -> sp.csr_matrix:
    """Same operator, assembled directly on the active set."""
    lin = np.asarray(lin, dtype=np.int64)
    m = lin.size
    n0, n1, n2 = (int(v) for v in n)
    i = lin // (n1 * n2)
    j = (lin // n2) % n1
    k = lin % n2
    w = [1.0 / (h[d] * h[d]) for d in range(3)]
    rows = [np.arange(m)]
    cols = [np.arange(m)]
    vals = [np.full(m, -2.0 * (w[0] + w[1] + w[2]))]
    for coord, extent, stride, wd in ((i, n0, n1 * n2, w[0]), (j, n1, n2, w[1]), (k, n2, 1, w[2])):
        for sgn in (-1, 1):
            inside = (coord + sgn >= 0) & (coord + sgn < extent)
            target = lin + sgn * stride
            pos = np.searchsorted(lin, target)
            pos_c = np.minimum(pos, m - 1)
            hit = inside & (pos < m) & (lin[pos_c] == target)
            rows.append(np.nonzero(hit)[0])
            cols.append(pos_c[hit])
            vals.append(np.full(int(hit.sum()), wd))
    L = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m, m))
    L.sum_duplicates()
    return (-0.5 * L).tocsr()


def laplacian_kron_19(n, h) -> sp.csr_matrix:
    """Full-box 19-point HOC Laplacian, eq. (B2), from Kronecker products."""
    D = [second_difference_1d(n[d], h[d]) for d in range(3)]
    I = [sp.identity(n[d], format="csr") for d in range(3)]

    def k3(a, b, c):
        return sp.kron(sp.kron(a, b), c)

    L = laplacian_kron(n, h)
    h2 = [h[d] * h[d] for d in range(3)]
    L = L + (1.0 / 12.0) * ((h2[0] + h2[1]) * k3(D[0], D[1], I[2]) + (h2[0] + h2[2]) * k3(D[0], I[1], D[2])
                            + (h2[1] + h2[2]) * k3(I[0], D[1], D[2]))
    return L.tocsr()


def kinetic_kron_19(n, h, lin: np.ndarray) -> sp.csr_matrix:
    """T~ from the 19-point stencil with the rows and columns outside the ROI removed."""
    L = laplacian_kron_19(n, h)
    lin = np.asarray(lin, dtype=np.int64)
    return (-0.5 * L[lin][:, lin]).tocsr()


def stencil_19_weights(h):
    """Weights of eq. (B2) by neighbour offset (di, dj, dk): the 1D second
    differences contribute 1/d^2 at the faces and -2/d^2 at the centre; each
    mixed term e_ab = (d_a^2 + d_b^2) / (12 d_a^2 d_b^2) times
    [1, -2, 1] (x) [1, -2, 1] contributes e_ab at the four edge points of the
    (a, b) plane, -2 e_ab at the four faces in that plane and 4 e_ab at the
    centre."""
    h2 = [h[d] * h[d] for d in range(3)]
    e = {}
    for a in range(3):
        for b in range(a + 1, 3):
            e[(a, b)] = (h2[a] + h2[b]) / (12.0 * h2[a] * h2[b])
    w = {}
    w[(0, 0, 0)] = sum(-2.0 / h2[d] for d in range(3)) + 4.0 * sum(e.values())
    for d in range(3):
        face = 1.0 / h2[d] - 2.0 * sum(v for (a, b), v in e.items() if d in (a, b))
        for sgn in (-1, 1):
            off = [0, 0, 0]
            off[d] = sgn
            w[tuple(off)] = face
    for (a, b), v in e.items():
        for sa in (-1, 1):
            for sb in (-1, 1):
                off = [0, 0, 0]
                off[a], off[b] = sa, sb
                w[tuple(off)] = v
    return w


def laplacian_kron_27(n, h) -> sp.csr_matrix:
    """Full-box cubic 27-point Laplacian for equal spacings h: (1/(30 h^2))
    [-128 I + 14 F + 3 E + C] with F, E, C the sums over the faces, edges and
    corners, built from Kronecker products of the 1D neighbour sum
    P = [1, 0, 1] (Dirichlet) and identities."""
    hh = float(h[0])
    if max(abs(h[1] - hh), abs(h[2] - hh)) > 1e-12 * hh:
        raise ValueError("the 27-point stencil is defined here for equal spacings")
    P = [sp.diags([np.ones(n[d] - 1), np.ones(n[d] - 1)], [-1, 1], shape=(n[d], n[d]), format="csr")
         for d in range(3)]
    I = [sp.identity(n[d], format="csr") for d in range(3)]

    def k3(a, b, c):
        return sp.kron(sp.kron(a, b), c)

    F = k3(P[0], I[1], I[2]) + k3(I[0], P[1], I[2]) + k3(I[0], I[1], P[2])
    E = k3(P[0], P[1], I[2]) + k3(P[0], I[1], P[2]) + k3(I[0], P[1], P[2])
    Cn = k3(P[0], P[1], P[2])
    Id = k3(I[0], I[1], I[2])
    return ((-128.0 * Id + 14.0 * F + 3.0 * E + Cn) / (30.0 * hh * hh)).tocsr()


def kinetic_kron_27(n, h, lin: np.ndarray) -> sp.csr_matrix:
    L = laplacian_kron_27(n, h)
    lin = np.asarray(lin, dtype=np.int64)
    return (-0.5 * L[lin][:, lin]).tocsr()


def stencil_27_weights(h):
    """Weights of the cubic 27-point stencil by offset, for equal spacings."""
    hh = float(h[0])
    w = {}
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for dk in (-1, 0, 1):
                nz = (di != 0) + (dj != 0) + (dk != 0)
                w[(di, dj, dk)] = {0: -128.0, 1: 14.0, 2: 3.0, 3: 1.0}[nz] / (30.0 * hh * hh)
    return w


def _kinetic_direct_weights(n, lin: np.ndarray, weights) -> sp.csr_matrix:
    lin = np.asarray(lin, dtype=np.int64)
    m = lin.size
    n0, n1, n2 = (int(v) for v in n)
    coords = (lin // (n1 * n2), (lin // n2) % n1, lin % n2)
    ext = (n0, n1, n2)
    strides = (n1 * n2, n2, 1)
    rows, cols, vals = [], [], []
    for off, wv in weights.items():
        inside = np.ones(m, bool)
        for d in range(3):
            inside &= (coords[d] + off[d] >= 0) & (coords[d] + off[d] < ext[d])
        target = lin + sum(off[d] * strides[d] for d in range(3))
        pos = np.searchsorted(lin, target)
        pos_c = np.minimum(pos, m - 1)
        hit = inside & (pos < m) & (lin[pos_c] == target)
        rows.append(np.nonzero(hit)[0])
        cols.append(pos_c[hit])
        vals.append(np.full(int(hit.sum()), wv))
    L = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m, m))
    L.sum_duplicates()
    return (-0.5 * L).tocsr()


def kinetic_direct_27(n, h, lin: np.ndarray) -> sp.csr_matrix:
    """The 27-point operator assembled directly on the active set."""
    return _kinetic_direct_weights(n, lin, stencil_27_weights(h))


def kinetic_direct_19(n, h, lin: np.ndarray) -> sp.csr_matrix:
    """The 19-point operator assembled directly on the active set."""
    return _kinetic_direct_weights(n, lin, stencil_19_weights(h))


def apply(T: sp.csr_matrix, psi: np.ndarray) -> np.ndarray:
    """T~ psi for complex psi; T~ is real, so it acts on Re and Im separately."""
    if np.iscomplexobj(psi):
        return T @ psi.real + 1j * (T @ psi.imag)
    return T @ psi
