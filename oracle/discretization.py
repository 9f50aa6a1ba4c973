"""Cell-centred finite-volume discretization of the zero-frequency diffusion model.

Section 2, eq. (PDE): -div(D grad eta) + mu eta = g on a box, eta = 0 on the
lateral faces, 0.25 eta + (D/2) d eta / d xi = 0 on the top/bottom faces.
The paper says only "finite difference"; the reading used here is a
symmetric cell-centred finite-volume scheme on a uniform grid of spacing
h = 1 / n_x (cells are cubes, the box is n_i * h long on axis i):

  interior face between cells c, c':  T = h^(d-2) * 2 D_c D_c' / (D_c + D_c')
  Dirichlet face (eta = 0 on it):      T = h^(d-2) * 2 D_c
  Robin face:                          T = h^(d-1) * 2 D_c / (h + 4 D_c)
  row c:  (A eta)_c = sum_interior T (eta_c - eta_c') + sum_boundary T eta_c
                      + h^d mu_c eta_c

The Robin coefficient follows from the face value eta_b = 4 D eta_c / (h + 4 D)
that satisfies the Robin condition with a half-cell one-sided difference,
and the outward flux 0.5 eta_b per unit face area.  A is symmetric positive
definite, so A^T = A (the adjoint solves of Section 3.3 use the same matrix).

Cells are numbered i + n_x (j + n_y k); arrays of cell values are shaped
(n_z, n_y, n_x) (3D) or (n_y, n_x) (2D) in C order, so ravel() gives that
numbering.  Boundary codes: 0 = Dirichlet, 1 = Robin, per face
(-x, +x, -y, +y, -z, +z).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def spacing(n) -> float:
    """Uniform grid spacing h = 1 / n_x."""
    return 1.0 / n[0]


def cell_shape(n) -> tuple:
    """numpy array shape of a cell field, slowest axis first."""
    return tuple(reversed(tuple(n)))


def cell_centres(n) -> np.ndarray:
    """(N, d) array of cell-centre coordinates (i + 1/2) h, in cell order."""
    h = spacing(n)
    d = len(n)
    axes = [(np.arange(n[a]) + 0.5) * h for a in range(d)]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")   # slowest axis first
    cols = [m.ravel() for m in reversed(mesh)]           # x, y, (z)
    return np.stack(cols, axis=1)


def _boundary_T(bc_code: int, Dc: np.ndarray, h: float, d: int) -> np.ndarray:
    if bc_code == 0:
        return h ** (d - 2) * 2.0 * Dc
    if bc_code == 1:
        return h ** (d - 1) * 2.0 * Dc / (h + 4.0 * Dc)
    raise ValueError(f"unknown boundary code {bc_code}")


def face_transmissibilities(n, bc, D: np.ndarray):
    """Interior face coefficients per axis and the boundary diagonal b0.

    Returns (T_int, b0): T_int[a] has the shape of the cell field with the
    last cell along axis a dropped (face between cell and its +a neighbour);
    b0 is the per-cell sum of boundary-face coefficients.
    """
    d = len(n)
    h = spacing(n)
    D = np.asarray(D, dtype=np.float64).reshape(cell_shape(n))
    T_int = []
    b0 = np.zeros_like(D)
    for a in range(d):
        ax = d - 1 - a                    # numpy axis of grid axis a
        lo = [slice(None)] * d
        hi = [slice(None)] * d
        lo[ax] = slice(0, n[a] - 1)
        hi[ax] = slice(1, n[a])
        Dl, Dh = D[tuple(lo)], D[tuple(hi)]
        T_int.append(h ** (d - 2) * 2.0 * Dl * Dh / (Dl + Dh))
        first = [slice(None)] * d
        last = [slice(None)] * d
        first[ax] = slice(0, 1)
        last[ax] = slice(n[a] - 1, n[a])
        b0[tuple(first)] += _boundary_T(bc[2 * a], D[tuple(first)], h, d)
        b0[tuple(last)] += _boundary_T(bc[2 * a + 1], D[tuple(last)], h, d)
    return T_int, b0


def assemble(n, bc, D: np.ndarray, mua: np.ndarray) -> sp.csr_matrix:
    """Sparse A(p) in CSR, FP64 (Section 2, eqs. PDE and compmeas with omega = 0)."""
    d = len(n)
    h = spacing(n)
    N = int(np.prod(n))
    T_int, b0 = face_transmissibilities(n, bc, D)
    idx = np.arange(N).reshape(cell_shape(n))
    diag = b0.ravel() + h ** d * np.asarray(mua, dtype=np.float64).ravel()
    rows, cols, vals = [], [], []
    for a in range(d):
        ax = d - 1 - a
        lo = [slice(None)] * d
        hi = [slice(None)] * d
        lo[ax] = slice(0, n[a] - 1)
        hi[ax] = slice(1, n[a])
        c0 = idx[tuple(lo)].ravel()
        c1 = idx[tuple(hi)].ravel()
        t = T_int[a].ravel()
        np.add.at(diag, c0, t)
        np.add.at(diag, c1, t)
        rows += [c0, c1]
        cols += [c1, c0]
        vals += [-t, -t]
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates()
    return A


def diffusion_from_mua(mua: np.ndarray, mus_prime: float) -> np.ndarray:
    """D = 1 / (3 (mu_a + mu_s')): the diffusion approximation's coefficient.

    Reading: D is evaluated once from the reference absorption and then held
    fixed (the paper treats D as known, Section 2), so dA/dp is diagonal.
    """
    return 1.0 / (3.0 * (np.asarray(mua, dtype=np.float64) + mus_prime))


def source_matrix(N: int, cells: np.ndarray) -> sp.csr_matrix:
    """B (or C): one unit column per optode, the unit integrated source in its cell."""
    cells = np.asarray(cells)
    k = cells.size
    return sp.csr_matrix((np.ones(k), (cells, np.arange(k))), shape=(N, k))
