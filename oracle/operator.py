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


def apply(T: sp.csr_matrix, psi: np.ndarray) -> np.ndarray:
    """T~ psi for complex psi; T~ is real, so it acts on Re and Im separately."""
    if np.iscomplexobj(psi):
        return T @ psi.real + 1j * (T @ psi.imag)
    return T @ psi
