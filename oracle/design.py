"""Optimized and complementary simultaneous sources/detectors (Section 3.2, Alg. 1).

The Jacobian is read as a third-order tensor with blocks J_j = J[j n_d:(j+1) n_d, :]
for source j (detector index fastest, as in Alg. 1 and eq. Jtensor).  The
optimized directions maximize ||(W^T kron V^T) J||_F^2 over isometric W (n_s x q_s)
and V (n_d x q_d) (eq. maxprob); they are found by the HOOI variant of
steps (1)-(3):
  (1) V <- leading q_d left singular vectors of J~ = [J_1 .. J_ns]   (eq. Jtilde)
  repeat
  (2) K~ = [K_1 .. K_qd], row j of K_l = v_l^T J_j;  W <- leading q_s left
      singular vectors of K~                                          (eq. Ktilde)
  (3) L~ = [L_1 .. L_qs], L_l = sum_j (w_l)_j J_j;   V <- leading q_d left
      singular vectors of L~                                          (eq. Ltilde)
  until the pair (V, W) stops changing.
Reading of the stopping rule ("sufficiently small"): the Frobenius norm of the
change of both orthogonal projectors V V^T and W W^T below tol (1e-10), or
50 iterations.

Complement (eqs. newW, newV): with [W_hat W_c] orthogonal,
W = [W_hat, W_c Y], Y = (l_s - q_s)^{-1/2} x Rademacher signs of shape
(n_s - q_s) x (l_s - q_s) (the paper's y_j in R^{l_s - q_s} is read as a typo
for R^{n_s - q_s}, since W_c has n_s - q_s columns).
"""

from __future__ import annotations

import numpy as np


def source_block(J: np.ndarray, n_d: int, j: int) -> np.ndarray:
    return J[j * n_d:(j + 1) * n_d, :]


def leading_left_singular_vectors(M: np.ndarray, q: int) -> np.ndarray:
    U, _, _ = np.linalg.svd(M, full_matrices=False)
    return U[:, :q]


def objective(J: np.ndarray, W: np.ndarray, V: np.ndarray) -> float:
    """||(W^T kron V^T) J||_F^2 (eq. maxprob)."""
    return float(np.sum((np.kron(W, V).T @ J) ** 2))


def unfold_J(J: np.ndarray, n_d: int, n_s: int) -> np.ndarray:
    """J~ of eq. (Jtilde): the source blocks side by side, n_d x (n_s n_p)."""
    return np.hstack([source_block(J, n_d, j) for j in range(n_s)])


def unfold_K(J: np.ndarray, n_d: int, n_s: int, V: np.ndarray) -> np.ndarray:
    """K~ of eq. (Ktilde), n_s x (q_d n_p)."""
    blocks = []
    for l in range(V.shape[1]):
        Kl = np.vstack([V[:, l] @ source_block(J, n_d, j) for j in range(n_s)])
        blocks.append(Kl)
    return np.hstack(blocks)


def unfold_L(J: np.ndarray, n_d: int, n_s: int, W: np.ndarray) -> np.ndarray:
    """L~ of eq. (Ltilde), n_d x (q_s n_p)."""
    blocks = []
    for l in range(W.shape[1]):
        Ll = np.zeros((n_d, J.shape[1]))
        for j in range(n_s):
            Ll += W[j, l] * source_block(J, n_d, j)
        blocks.append(Ll)
    return np.hstack(blocks)


def hooi(J: np.ndarray, n_d: int, n_s: int, q_d: int, q_s: int, tol: float = 1e-10,
         maxit: int = 50):
    """Alg. 1.  Returns (W_hat, V_hat, objective history, iterations)."""
    V = leading_left_singular_vectors(unfold_J(J, n_d, n_s), q_d)
    W = None
    history = []
    it = 0
    for it in range(1, maxit + 1):
        W_new = leading_left_singular_vectors(unfold_K(J, n_d, n_s, V), q_s)
        V_new = leading_left_singular_vectors(unfold_L(J, n_d, n_s, W_new), q_d)
        history.append(objective(J, W_new, V_new))
        dV = np.linalg.norm(V_new @ V_new.T - V @ V.T)
        dW = np.inf if W is None else np.linalg.norm(W_new @ W_new.T - W @ W.T)
        V, W = V_new, W_new
        if dV < tol and dW < tol:
            break
    return W, V, history, it


def orthonormal_complement(What: np.ndarray) -> np.ndarray:
    """W_c with [W_hat W_c] orthogonal, from a complete QR factorization."""
    Q, _ = np.linalg.qr(What, mode="complete")
    return Q[:, What.shape[1]:]


def complemented_sample(What: np.ndarray, Wc: np.ndarray, signs: np.ndarray) -> np.ndarray:
    """W = [W_hat, W_c Y] with Y = (l - q)^{-1/2} signs (eqs. newW, newV)."""
    signs = np.asarray(signs, dtype=np.float64)
    Y = signs / np.sqrt(signs.shape[1]) if signs.shape[1] > 0 else signs
    return np.hstack([What, Wc @ Y])


def lift(W: np.ndarray, Wt: np.ndarray) -> np.ndarray:
    """Orthonormal basis of range(W Wt): optimized directions found on the sampled
    tensor, expressed in the full source (detector) space."""
    Q, _ = np.linalg.qr(W @ Wt)
    return Q


def thin_svd(Js: np.ndarray):
    """J_s = U diag(s) Y^T, economy size (the SVD behind the Gauss-Newton model, eq. GN)."""
    return np.linalg.svd(Js, full_matrices=False)


def tsvd_step(Js: np.ndarray, r: np.ndarray, t: int) -> np.ndarray:
    """Truncated-SVD Gauss-Newton step for min ||J_s d + r_s|| (eqs. Eq:NLLS,
    TREGS J), kept to the t largest singular values (the directions the
    regularized model favours): d = -sum_{i < t} (u_i^T r / s_i) y_i."""
    U, s, Yt = np.linalg.svd(np.asarray(Js), full_matrices=False)
    c = (U[:, :t].T @ np.asarray(r)) / s[:t]
    return -(Yt[:t].T @ c)
