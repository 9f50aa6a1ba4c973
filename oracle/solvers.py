"""Reference linear solvers for A(p) X = RHS.

Section 3.3 allows "iterative solvers or sparse direct solvers depending on
the size of the system".  The oracle offers both, written plainly:
  * LAPACK banded Cholesky (A is SPD with half-bandwidth n_x n_y in 3D,
    n_x in 2D) for exact fields on small grids;
  * SuperLU as an independent direct cross-check;
  * textbook Jacobi-preconditioned CG, one column at a time, x0 = 0, stopped
    when ||b - A x||_2 / ||b||_2 <= rtol on the recursively updated residual.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def half_bandwidth(n) -> int:
    return int(np.prod(n[:-1]))


def banded_cholesky_solve(A: sp.spmatrix, RHS: np.ndarray, n) -> np.ndarray:
    """Solve A X = RHS by Cholesky factorization of A stored in LAPACK upper band form."""
    u = half_bandwidth(n)
    N = A.shape[0]
    ab = np.zeros((u + 1, N))
    A = sp.csr_matrix(A)
    for k in range(u + 1):
        dk = A.diagonal(k)
        ab[u - k, k:] = dk
    cb = sla.cholesky_banded(ab, lower=False)
    return sla.cho_solve_banded((cb, False), np.asarray(RHS, dtype=np.float64))


def splu_solve(A: sp.spmatrix, RHS: np.ndarray) -> np.ndarray:
    lu = spla.splu(sp.csc_matrix(A))
    RHS = np.asarray(RHS, dtype=np.float64)
    return lu.solve(RHS)


def direct_solve(A: sp.spmatrix, RHS: np.ndarray, n) -> np.ndarray:
    """Banded Cholesky when the band fits comfortably, SuperLU otherwise."""
    N = A.shape[0]
    if N * (half_bandwidth(n) + 1) <= 2.0e7:
        return banded_cholesky_solve(A, RHS, n)
    return splu_solve(A, RHS)


def pcg_jacobi(A: sp.spmatrix, b: np.ndarray, rtol: float, maxiter: int = 100000):
    """Jacobi-PCG for one right-hand side.  Returns (x, iterations, relres).

    iterations counts applications of A to a search direction; relres is the
    recursively updated ||r|| / ||b|| at exit.
    """
    A = sp.csr_matrix(A)
    b = np.asarray(b, dtype=np.float64)
    dinv = 1.0 / A.diagonal()
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    relres = 1.0
    while it < maxiter:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        relres = np.linalg.norm(r) / bnorm
        if relres <= rtol:
            break
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, relres


def pcg_jacobi_multi(A: sp.spmatrix, RHS: np.ndarray, rtol: float, maxiter: int = 100000):
    """Column-by-column Jacobi-PCG.  Returns (X, iterations[k], relres[k])."""
    RHS = np.asarray(RHS, dtype=np.float64)
    X = np.zeros_like(RHS)
    its = np.zeros(RHS.shape[1], dtype=np.int64)
    rel = np.zeros(RHS.shape[1])
    for j in range(RHS.shape[1]):
        X[:, j], its[j], rel[j] = pcg_jacobi(A, RHS[:, j], rtol, maxiter)
    return X, its, rel


def relative_residuals(A: sp.spmatrix, X: np.ndarray, RHS: np.ndarray) -> np.ndarray:
    """True per-column ||RHS - A X||_2 / ||RHS||_2, recomputed with the CSR matrix."""
    R = np.asarray(RHS) - A @ np.asarray(X)
    bn = np.linalg.norm(RHS, axis=0)
    bn = np.where(bn == 0.0, 1.0, bn)
    return np.linalg.norm(R, axis=0) / bn
