"""Randomized optimized sources and detectors without the full Jacobian
(Section 3.2, the remark on computing the optimized directions from a cheap
randomized low-rank approximation of J; Section 5).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Alg. 1 needs the leading left singular vectors of three unfoldings of the
Jacobian tensor cal-J_{m j k} = c_m^T A^-1 (dA/dp_k) A^-1 b_j (detector m,
source j, parameter k; eq. Jtensor, written without the minus sign of
eq. Jacobiancomp as in Alg. 1):
  J~ (n_d x n_s n_p), K~ = [K_1 .. K_qd] (n_s x q_d n_p), L~ (n_d x q_s n_p).
Reading (the passage is garbled in the source; it names a randomized
low-rank approximation in the sense of Halko, Martinsson and Tropp): each
unfolding M is replaced by a sketch Y = M Omega whose k test vectors are
Khatri-Rao products omega = x kron theta, x a Rademacher vector over the
sources (for J~) or a Gaussian vector over the q columns of the current
W~ or V~ (for L~, K~), theta a standard Gaussian vector over the parameters.
Then E[omega omega^T] = I, so Y Y^T / k estimates the Gram M M^T without
bias (the trace-estimator idea the paper's sampled misfit rests on), and
the leading left singular vectors of Y stand in for those of M.  Each test
vector costs one forward and one adjoint solve instead of n_s + n_d for J:
  J~ (w kron theta)  = C^T A^-1 (dA/d theta) A^-1 B w,
  K~ (a kron theta)  = B^T A^-T (dA/d theta) A^-T C V~ a,
  L~ (a kron theta)  = C^T A^-1 (dA/d theta) A^-1 B W~ a,
with dA/d theta = sum_k theta_k dA/dp_k.  The sketched HOOI takes step (1)
once and steps (2)-(3) a fixed number of sweeps (fresh test vectors each
time, so the projector-change stopping rule of Alg. 1 does not apply).

Here the sketches are formed from their definition, as contractions of the
full Jacobian; the matrix-free route with two solves per test vector is
`sketch_matrix_free`, pinned against the definition in the tests.
"""

from __future__ import annotations

import numpy as np

from . import estimators as est
from . import solvers


def _blocks(J: np.ndarray, n_d: int, n_s: int):
    """cal-J as an (n_d, n_s, n_p) array from J (rows j + n_d i, minus sign)."""
    n_p = J.shape[1]
    return -np.asarray(J).reshape(n_s, n_d, n_p).transpose(1, 0, 2)


def det_sketch(J: np.ndarray, n_d: int, n_s: int, X: np.ndarray, Th: np.ndarray) -> np.ndarray:
    """Columns sum_j X[j, l] cal-J[:, j, :] Th[:, l] (n_d x k): J~ or L~ times
    Khatri-Rao test vectors (X over sources)."""
    T = _blocks(J, n_d, n_s)
    k = X.shape[1]
    Y = np.zeros((n_d, k))
    for l in range(k):
        for j in range(n_s):
            Y[:, l] += X[j, l] * (T[:, j, :] @ Th[:, l])
    return Y


def src_sketch(J: np.ndarray, n_d: int, n_s: int, Ydet: np.ndarray, Th: np.ndarray) -> np.ndarray:
    """Columns [Ydet[:, l]^T cal-J[:, j, :] Th[:, l]]_j (n_s x k): K~ times
    Khatri-Rao test vectors (Ydet over detectors)."""
    T = _blocks(J, n_d, n_s)
    k = Ydet.shape[1]
    Y = np.zeros((n_s, k))
    for l in range(k):
        for j in range(n_s):
            Y[j, l] = Ydet[:, l] @ (T[:, j, :] @ Th[:, l])
    return Y


def leading(Y: np.ndarray, q: int) -> np.ndarray:
    U, _, _ = np.linalg.svd(Y, full_matrices=False)
    return U[:, :q]


def randomized_hooi(J: np.ndarray, n_d: int, n_s: int, q_d: int, q_s: int, draws: dict):
    """Sketched Alg. 1.  draws: 'w1' (n_s x k Rademacher), 't1' (n_p x k), and
    per sweep s: 'a2'[s] (q_d x k), 't2'[s], 'a3'[s] (q_s x k), 't3'[s]
    (Gaussian).  Returns (W~, V~, sketches)."""
    sk = {"Y1": det_sketch(J, n_d, n_s, draws["w1"], draws["t1"])}
    V = leading(sk["Y1"], q_d)
    W = None
    for s in range(len(draws["a2"])):
        Y2 = src_sketch(J, n_d, n_s, V @ draws["a2"][s], draws["t2"][s])
        W = leading(Y2, q_s)
        Y3 = det_sketch(J, n_d, n_s, W @ draws["a3"][s], draws["t3"][s])
        V = leading(Y3, q_d)
        sk[f"Y2_{s}"], sk[f"Y3_{s}"] = Y2, Y3
    return W, V, sk


def sketch_solves(k: int, sweeps: int) -> int:
    """Large solves of the sketched design: one forward and one adjoint solve
    per test vector, k test vectors per sketch, 1 + 2 sweeps sketches."""
    return 2 * k * (1 + 2 * sweeps)


def sketch_matrix_free(A, n, N: int, src_cells, det_cells, G: np.ndarray, X: np.ndarray,
                       Th: np.ndarray, side: str) -> np.ndarray:
    """The same sketches with two direct solves per test vector:
    side 'det': C^T A^-1 diag(G Th_l) A^-1 B X_l;  side 'src':
    B^T A^-T diag(G Th_l) A^-T C X_l (G: N x n_p, h^d d mu / d p)."""
    k = X.shape[1]
    if side == "det":
        F = solvers.direct_solve(A, est.simultaneous_rhs(N, src_cells, X), n)
        S = solvers.direct_solve(A.T.tocsr(), (G @ Th) * F, n)
        return S[np.asarray(det_cells), :]
    F = solvers.direct_solve(A.T.tocsr(), est.simultaneous_rhs(N, det_cells, X), n)
    S = solvers.direct_solve(A, (G @ Th) * F, n)
    assert S.shape[1] == k
    return S[np.asarray(src_cells), :]
