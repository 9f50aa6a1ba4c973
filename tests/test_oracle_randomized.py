"""Pins of the sketched Alg. 1 (oracle/randomized.py).

  * unbiasedness: over every Rademacher source vector w and every
    parameter vector theta of an isotropic design (+-sqrt(n_p) e_k), the mean
    of y y^T with y = J~ (w kron theta) is exactly J~ J~^T (the same
    trace-estimator identity as Thm 3.1);
  * exact recovery: for a Jacobian tensor of multilinear rank (q_d, q_s) in
    the detector and source modes, any k >= q test vectors reproduce the
    projectors of the exact Alg. 1;
  * the matrix-free sketches (one forward and one adjoint direct solve per
    test vector) equal the definition, contractions of the full Jacobian of
    the PDE, on a small 3D grid, for both kinds of sketch;
  * the solve count 2 k (1 + 2 sweeps).
"""

import itertools

import numpy as np
import pytest

import synthetic
from oracle import design
from oracle import estimators as est
from oracle import problem as oprob
from oracle import randomized as rnd
from oracle import solvers


def _J_from_tensor(T):
    """J (rows j + n_d i, minus sign) from cal-J[m, j, k]."""
    n_d, n_s, n_p = T.shape
    return -T.transpose(1, 0, 2).reshape(n_s * n_d, n_p)


def test_sketch_gram_is_unbiased():
    rng = np.random.default_rng(3)
    n_d, n_s, n_p = 3, 4, 5
    T = rng.standard_normal((n_d, n_s, n_p))
    J = _J_from_tensor(T)
    Jt = design.unfold_J(-J, n_d, n_s)           # J~ of eq. Jtilde (n_d x n_s n_p)
    acc = np.zeros((n_d, n_d))
    count = 0
    for w in itertools.product((-1.0, 1.0), repeat=n_s):
        for kk in range(n_p):
            for sgn in (-1.0, 1.0):
                th = np.zeros(n_p)
                th[kk] = sgn * np.sqrt(n_p)
                y = rnd.det_sketch(J, n_d, n_s, np.array(w)[:, None], th[:, None])[:, 0]
                acc += np.outer(y, y)
                count += 1
    assert np.allclose(acc / count, Jt @ Jt.T, rtol=1e-12, atol=1e-12)


def test_exact_recovery_at_low_multilinear_rank():
    rng = np.random.default_rng(4)
    n_d, n_s, n_p, q_d, q_s, k = 9, 11, 7, 2, 3, 5
    V0 = np.linalg.qr(rng.standard_normal((n_d, q_d)))[0]
    W0 = np.linalg.qr(rng.standard_normal((n_s, q_s)))[0]
    core = rng.standard_normal((q_d, q_s, n_p))
    T = np.einsum("ma,jb,abk->mjk", V0, W0, core)
    J = _J_from_tensor(T)
    We, Ve, _, _ = design.hooi(J, n_d, n_s, q_d, q_s)
    draws = {"w1": rng.choice([-1.0, 1.0], size=(n_s, k)), "t1": rng.standard_normal((n_p, k)),
             "a2": [rng.standard_normal((q_d, k))], "t2": [rng.standard_normal((n_p, k))],
             "a3": [rng.standard_normal((q_s, k))], "t3": [rng.standard_normal((n_p, k))]}
    Wr, Vr, _ = rnd.randomized_hooi(J, n_d, n_s, q_d, q_s, draws)
    assert np.linalg.norm(Wr @ Wr.T - We @ We.T) <= 1e-10
    assert np.linalg.norm(Vr @ Vr.T - Ve @ Ve.T) <= 1e-10
    assert np.linalg.norm(Vr @ Vr.T - V0 @ V0.T) <= 1e-10


def test_matrix_free_sketches_equal_the_definition():
    wl = synthetic.make_workload(synthetic.get_config("inv_t", n=(12, 12, 10),
                                                      src_lattice=(3, 3), det_lattice=(3, 2)))
    prob = oprob.build(wl)
    th = wl.theta_ref
    A = prob.operator(th)
    G = prob.G(th)
    n_s, n_d = len(wl.src_cells), len(wl.det_cells)
    U = solvers.direct_solve(A, est.simultaneous_rhs(prob.N, wl.src_cells, np.eye(n_s)), prob.n)
    Z = solvers.direct_solve(A.T.tocsr(), est.simultaneous_rhs(prob.N, wl.det_cells, np.eye(n_d)),
                             prob.n)
    J = est.jacobian_sparse_loops(U, Z, G)
    rng = np.random.default_rng(5)
    k = 4
    X = rng.choice([-1.0, 1.0], size=(n_s, k))
    Yd = rng.standard_normal((n_d, k))
    Th = rng.standard_normal((G.shape[1], k))
    a = rnd.det_sketch(J, n_d, n_s, X, Th)
    b = rnd.sketch_matrix_free(A, prob.n, prob.N, wl.src_cells, wl.det_cells, G, X, Th, "det")
    assert np.allclose(a, b, rtol=1e-10, atol=1e-12 * np.abs(a).max())
    c = rnd.src_sketch(J, n_d, n_s, Yd, Th)
    d = rnd.sketch_matrix_free(A, prob.n, prob.N, wl.src_cells, wl.det_cells, G, Yd, Th, "src")
    assert np.allclose(c, d, rtol=1e-10, atol=1e-12 * np.abs(c).max())


def test_sketch_solve_count():
    assert rnd.sketch_solves(8, 2) == 80
    assert rnd.sketch_solves(4, 0) == 8
