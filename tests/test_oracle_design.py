"""Pins for Alg. 1 (optimized sources/detectors) and the complementary construction.

* with one parameter and q_s = q_d = q, maximizing ||V^T M W||_F over
  isometric V, W gives the sum of the q largest squared singular values of M
  (Ky Fan), so HOOI must reach numpy's SVD value;
* Thm. 3.2: if J = (W0 kron V0) G0 with isometric W0, V0, one iteration of
  steps (1)-(3) preserves ||J||_F exactly;
* the HOOI objective never decreases;
* [W_hat W_c] is orthogonal; Thm. 3.3 (E[W W^T] = I and E ||V^T R W||^2 =
  ||R||^2 for the complemented samples) by exact enumeration of the signs.
"""

import itertools

import numpy as np
import pytest

from oracle import design, estimators as est


def _isometric(rng, n, q):
    Q, _ = np.linalg.qr(rng.standard_normal((n, q)))
    return Q


@pytest.mark.parametrize("q", [1, 2, 3])
def test_single_parameter_reduces_to_ky_fan(q):
    rng = np.random.default_rng(10 + q)
    n_d, n_s = 7, 6
    M = rng.standard_normal((n_d, n_s))
    J = M.reshape(-1, 1, order="F")            # row det + n_d * src
    W, V, hist, _ = design.hooi(J, n_d, n_s, q, q)
    s = np.linalg.svd(M, compute_uv=False)
    assert hist[-1] == pytest.approx(np.sum(s[:q] ** 2), rel=1e-12)
    assert np.allclose(W.T @ W, np.eye(q), atol=1e-13)
    assert np.allclose(V.T @ V, np.eye(q), atol=1e-13)


@pytest.mark.parametrize("q_s,q_d", [(1, 1), (2, 3), (3, 2)])
def test_theorem_3_2_one_iteration_exact(q_s, q_d):
    rng = np.random.default_rng(20 + q_s * 3 + q_d)
    n_s, n_d, n_p = 9, 8, 5
    W0, V0 = _isometric(rng, n_s, q_s), _isometric(rng, n_d, q_d)
    G0 = rng.standard_normal((q_s * q_d, n_p))
    J = np.kron(W0, V0) @ G0
    W, V, hist, its = design.hooi(J, n_d, n_s, q_d, q_s, maxit=1)
    assert hist[0] == pytest.approx(np.sum(J ** 2), rel=1e-12)
    assert np.linalg.norm(W @ W.T - W0 @ W0.T) < 1e-10
    assert np.linalg.norm(V @ V.T - V0 @ V0.T) < 1e-10


def test_objective_monotone_and_converges():
    rng = np.random.default_rng(30)
    n_s, n_d, n_p = 10, 9, 12
    J = rng.standard_normal((n_s * n_d, n_p))
    W, V, hist, its = design.hooi(J, n_d, n_s, 2, 3, tol=1e-10, maxit=200)
    assert np.all(np.diff(hist) >= -1e-12 * hist[-1])
    assert its < 200
    assert hist[-1] <= np.sum(J ** 2)
    assert hist[-1] == pytest.approx(design.objective(J, W, V), rel=1e-14)


def test_complement_orthogonal():
    rng = np.random.default_rng(40)
    What = _isometric(rng, 12, 3)
    Wc = design.orthonormal_complement(What)
    assert Wc.shape == (12, 9)
    assert np.allclose(What.T @ Wc, 0.0, atol=1e-14)
    assert np.allclose(Wc.T @ Wc, np.eye(9), atol=1e-14)
    assert np.allclose(What @ What.T + Wc @ Wc.T, np.eye(12), atol=1e-14)


def test_theorem_3_3_exact_enumeration():
    rng = np.random.default_rng(50)
    n_s, q_s, l_s = 4, 1, 3
    n_d, q_d, l_d = 3, 1, 2
    What, Vhat = _isometric(rng, n_s, q_s), _isometric(rng, n_d, q_d)
    Wc, Vc = design.orthonormal_complement(What), design.orthonormal_complement(Vhat)
    R = rng.standard_normal((n_d, n_s))
    EW = np.zeros((n_s, n_s))
    EV = np.zeros((n_d, n_d))
    Ef = 0.0
    count = 0
    for ys in itertools.product((-1, 1), repeat=(n_s - q_s) * (l_s - q_s)):
        Y = np.array(ys).reshape(n_s - q_s, l_s - q_s)
        W = design.complemented_sample(What, Wc, Y)
        EW += W @ W.T
        for zs in itertools.product((-1, 1), repeat=(n_d - q_d) * (l_d - q_d)):
            Zs = np.array(zs).reshape(n_d - q_d, l_d - q_d)
            V = design.complemented_sample(Vhat, Vc, Zs)
            Ef += np.sum((V.T @ R @ W) ** 2)
            if ys == (1,) * len(ys):
                pass
            count += 1
    n_z = 2 ** ((n_d - q_d) * (l_d - q_d))
    for zs in itertools.product((-1, 1), repeat=(n_d - q_d) * (l_d - q_d)):
        V = design.complemented_sample(Vhat, Vc, np.array(zs).reshape(n_d - q_d, l_d - q_d))
        EV += V @ V.T
    assert np.allclose(EW / (count / n_z), np.eye(n_s), atol=1e-13)
    assert np.allclose(EV / n_z, np.eye(n_d), atol=1e-13)
    assert Ef / count == pytest.approx(np.sum(R ** 2), rel=1e-13)


def test_lift_and_thin_svd():
    rng = np.random.default_rng(60)
    W = est.sample_matrix(rng.choice([-1, 1], size=(16, 5)))
    Wt = _isometric(rng, 5, 2)
    Q = design.lift(W, Wt)
    assert np.allclose(Q.T @ Q, np.eye(2), atol=1e-14)
    P = W @ Wt
    assert np.allclose(Q @ (Q.T @ P), P, atol=1e-13)
    Js = rng.standard_normal((12, 30))
    U, s, Yt = design.thin_svd(Js)
    assert np.allclose((U * s) @ Yt, Js, atol=1e-13)


@pytest.mark.parametrize("shape", [(30, 12), (12, 30)])
def test_tsvd_step_full_rank_is_least_squares(shape):
    """All singular values kept: the minimum-norm least-squares solution of
    J d = -r (numpy.linalg.lstsq), tall and wide."""
    rng = np.random.default_rng(sum(shape))
    J = rng.standard_normal(shape)
    r = rng.standard_normal(shape[0])
    d = design.tsvd_step(J, r, min(shape))
    ref = -np.linalg.lstsq(J, r, rcond=None)[0]
    assert np.allclose(d, ref, atol=1e-12)


def test_tsvd_step_truncated_residual_orthogonal_to_kept_directions():
    """With t < rank the step lies in the span of the first t right vectors
    and the model residual J d + r has no component along the first t left
    vectors."""
    rng = np.random.default_rng(3)
    J = rng.standard_normal((25, 10)) @ np.diag(np.logspace(0, -6, 10))
    r = rng.standard_normal(25)
    t = 4
    d = design.tsvd_step(J, r, t)
    U, s, Yt = np.linalg.svd(J, full_matrices=False)
    assert np.linalg.norm(U[:, :t].T @ (J @ d + r)) <= 1e-12 * np.linalg.norm(r)
    assert np.linalg.norm(Yt[t:] @ d) <= 1e-12 * np.linalg.norm(d)
