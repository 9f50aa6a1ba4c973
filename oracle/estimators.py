"""Simultaneous sources/detectors, sampled misfit, sampled Jacobian and gradient.

Section 3.1 and Section 3.3.  Conventions:
  R = C^T A^{-1} B - D  (n_d x n_s), r = vec(R) column-major (eq. MartixR);
  W = l_s^{-1/2} [w_1 .. w_ls], V = l_d^{-1/2} [v_1 .. v_ld] (eqs. defW, defV);
  forward fields  U = A^{-1} (B W)   (N x l_s), the paper's z_i;
  adjoint fields  Z = A^{-T} (C V)   (N x l_d), the paper's y_j;
  sampled residual R_s = V^T (C^T U - D W) (l_d x l_s) (eq. EsTResidual);
  sampled Jacobian J_s = (W^T kron V^T) J, row (det j) + l_d * (src i), with
  J_s[j + l_d i, k] = - y_j^T (dA/dp_k) z_i (eq. Jacobian kth column, with
  the minus sign of eq. Jacobiancomp), dA/dp_k = diag(h^d d mu / d p_k).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import solvers


def sample_matrix(signs: np.ndarray) -> np.ndarray:
    """Rademacher sample matrix scaled by l^{-1/2} (eqs. defW, defV)."""
    signs = np.asarray(signs, dtype=np.float64)
    return signs / np.sqrt(signs.shape[1])


def simultaneous_rhs(N: int, cells: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """B W (or C V) as a dense N x l array: column l is sum_i W[i, l] e_{cell_i} (eq. Rw)."""
    weights = np.asarray(weights, dtype=np.float64)
    out = np.zeros((N, weights.shape[1]))
    for i, c in enumerate(np.asarray(cells)):
        out[c, :] += weights[i, :]
    return out


def measurements(A: sp.spmatrix, n, src_cells, det_cells) -> np.ndarray:
    """M = C^T A^{-1} B, n_d x n_s (eq. compmeas at omega = 0)."""
    N = A.shape[0]
    B = simultaneous_rhs(N, src_cells, np.eye(len(src_cells)))
    X = solvers.direct_solve(A, B, n)
    return X[np.asarray(det_cells), :]


def noisy_data(M_true: np.ndarray, xi: np.ndarray, level: float) -> np.ndarray:
    """Synthetic data with relative white noise of the given level (Section 4: 0.1%)."""
    return M_true * (1.0 + level * np.asarray(xi))


def sampled_residual(U: np.ndarray, det_cells, V: np.ndarray, DW: np.ndarray) -> np.ndarray:
    """R_s = V^T (C^T U - D W), l_d x l_s (eq. EsTResidual)."""
    CtU = np.asarray(U)[np.asarray(det_cells), :]
    return np.asarray(V).T @ (CtU - np.asarray(DW))


def misfit(Rs: np.ndarray) -> float:
    """f = 1/2 ||R_s||_F^2 (eqs. NonLeastSq1, TREGS J)."""
    return 0.5 * float(np.sum(np.asarray(Rs) ** 2))


def jacobian_loops(U: np.ndarray, Z: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Sampled Jacobian by an explicit loop nest over (source i, detector j, parameter k).

    G is the N x n_p matrix h^d d mu / d p (the diagonal of dA/dp_k in column k).
    """
    N, ls = U.shape
    ld = Z.shape[1]
    n_p = G.shape[1]
    J = np.empty((ls * ld, n_p))
    for i in range(ls):
        for j in range(ld):
            zy = U[:, i] * Z[:, j]
            for k in range(n_p):
                J[j + ld * i, k] = -np.dot(zy, G[:, k])
    return J


def jacobian_sparse_loops(U: np.ndarray, Z: np.ndarray, G: np.ndarray) -> np.ndarray:
    """The same loop nest visiting only the nonzeros of each column of G (Section 3.3,
    last paragraph: only the nonzero entries of dA/dp_k are referenced)."""
    ls, ld = U.shape[1], Z.shape[1]
    J = np.zeros((ls * ld, G.shape[1]))
    for k in range(G.shape[1]):
        nz = np.nonzero(G[:, k])[0]
        if nz.size == 0:
            continue
        g = G[nz, k]
        Uk, Zk = U[nz, :], Z[nz, :]
        for i in range(ls):
            for j in range(ld):
                J[j + ld * i, k] = -np.dot(Uk[:, i] * Zk[:, j], g)
    return J


def gradient_via_jacobian(Js: np.ndarray, Rs: np.ndarray) -> np.ndarray:
    """g = J_s^T vec(R_s) (the sampled gradient of eq. UnbiasedGrad)."""
    return np.asarray(Js).T @ np.asarray(Rs).reshape(-1, order="F")


def gradient_adjoint(U: np.ndarray, Z: np.ndarray, Rs: np.ndarray, G: np.ndarray) -> np.ndarray:
    """The same gradient without forming J_s.

    sum_{i,j} R_s[j,i] J_s[j + l_d i, k] = - sum_c G_ck sum_i U_ci (Z R_s)_ci.
    """
    Lam = np.asarray(Z) @ np.asarray(Rs)          # A^{-T} C V R_s
    s = np.sum(np.asarray(U) * Lam, axis=1)
    return -np.asarray(G).T @ s

