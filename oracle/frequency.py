"""Frequency-domain model (Section 2, eq. PDE with omega > 0; eq. compmeas and
its footnote; the footnote of Section 3.1 on several frequencies).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading: in the cell-centred finite-volume scheme the frequency term
i omega / nu eta integrates over a cell like the absorption term, so the
discrete matrix is A_w = A(p) + i kappa h^d I with kappa = omega / nu (the
paper's E is the identity except for zero rows at boundary nodes of its
vertex-centred scheme; this scheme has no unknowns on the boundary).  A_w
is complex symmetric (A_w^T = A_w), so the adjoint fields solve the same
system.  Measurements are complex, m = C^T A_w^-1 b, and the residual is
split into its real and imaginary parts (the footnote to eq. compmeas):
r = [Re vec(R); Im vec(R)], f = 1/2 (||Re R||^2 + ||Im R||^2).  dA_w/dp_k
= dA/dp_k (E does not depend on p), so the sampled Jacobian is
J_s[j + l_d i, k] = - sum_c G_ck Z_cj U_ci with complex U = A_w^-1 B W,
Z = A_w^-1 C V (no conjugation), stacked as [Re J_s; Im J_s].
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import estimators as est


def operator(prob, theta: np.ndarray, kappa: float) -> sp.csr_matrix:
    """A(theta) + i kappa h^d I."""
    A = prob.operator(theta).astype(np.complex128)
    return (A + 1j * kappa * prob.h ** prob.d * sp.identity(prob.N, format="csr")).tocsr()


def direct_solve(Aw: sp.spmatrix, RHS: np.ndarray) -> np.ndarray:
    """SuperLU on the complex matrix."""
    return spla.splu(sp.csc_matrix(Aw)).solve(np.asarray(RHS, dtype=np.complex128))


def relative_residuals(Aw: sp.spmatrix, X: np.ndarray, B: np.ndarray) -> np.ndarray:
    """||b_j - A_w x_j||_2 / ||b_j||_2 per column (conjugated norms)."""
    R = np.asarray(B) - Aw @ np.asarray(X)
    return np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)


def measurements(prob, wl, theta: np.ndarray, kappa: float) -> np.ndarray:
    """M = C^T A_w^-1 B (n_d x n_s, complex)."""
    Aw = operator(prob, theta, kappa)
    B = est.simultaneous_rhs(prob.N, wl.src_cells, np.eye(len(wl.src_cells)))
    return direct_solve(Aw, B)[np.asarray(wl.det_cells), :]


def evaluate(prob, wl, theta, kappa, W, V, data):
    """Complex fields, sampled residual, misfit, sampled Jacobian (complex and
    stacked real) and gradient at theta."""
    Aw = operator(prob, theta, kappa)
    U = direct_solve(Aw, est.simultaneous_rhs(prob.N, wl.src_cells, W))
    Z = direct_solve(Aw, est.simultaneous_rhs(prob.N, wl.det_cells, V))
    Rs = np.asarray(V).T @ (U[np.asarray(wl.det_cells), :] - np.asarray(data) @ np.asarray(W))
    f = 0.5 * float(np.sum(Rs.real ** 2) + np.sum(Rs.imag ** 2))
    G = prob.G(theta)
    ls, ld = U.shape[1], Z.shape[1]
    Jc = np.zeros((ls * ld, G.shape[1]), dtype=np.complex128)
    for k in range(G.shape[1]):
        nz = np.nonzero(G[:, k])[0]
        for i in range(ls):
            for j in range(ld):
                Jc[j + ld * i, k] = -np.sum(G[nz, k] * Z[nz, j] * U[nz, i])
    J = np.vstack([Jc.real, Jc.imag])
    r = np.concatenate([Rs.real.reshape(-1, order="F"), Rs.imag.reshape(-1, order="F")])
    return dict(Aw=Aw, U=U, Z=Z, Rs=Rs, f=f, Jc=Jc, J=J, r=r, g=J.T @ r, G=G)
