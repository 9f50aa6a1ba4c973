"""Pins for the oracle's linear solvers and forward model.

* banded Cholesky, SuperLU and the DST-II closed form agree;
* Jacobi-PCG reaches its tolerance and matches the direct solution;
* reciprocity: with co-located sources and detectors and A = A^T, the
  measurement matrix M = C^T A^{-1} B is symmetric (Section 2, eq. compmeas);
* linearity of simultaneous sources: A^{-1}(B W) = (A^{-1} B) W (eq. Rw).
"""

import numpy as np
import pytest

import synthetic
from oracle import discretization as disc
from oracle import estimators as est
from oracle import problem, solvers


def _dirichlet_const(n):
    N = int(np.prod(n))
    return disc.assemble(n, (0,) * (2 * len(n)), np.full(N, 0.3), np.full(N, 0.02))


@pytest.mark.parametrize("n", [(11, 9), (6, 7, 5)])
def test_direct_solvers_agree(n):
    A = _dirichlet_const(n)
    rng = np.random.default_rng(5)
    B = rng.standard_normal((A.shape[0], 3))
    x1 = solvers.banded_cholesky_solve(A, B, n)
    x2 = solvers.splu_solve(A, B)
    assert np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x2)


def test_pcg_matches_direct():
    wl = synthetic.make_workload(synthetic.get_config("t3d"))
    prob = problem.build(wl)
    A = prob.operator(wl.theta_ref)
    W = est.sample_matrix(wl.w_signs)
    BW = est.simultaneous_rhs(prob.N, wl.src_cells, W)
    X, its, rel = solvers.pcg_jacobi_multi(A, BW, 1e-12)
    assert np.all(rel <= 1e-12) and np.all(its > 5)
    true_rel = solvers.relative_residuals(A, X, BW)
    assert np.all(true_rel <= 1e-11)
    Xd = solvers.direct_solve(A, BW, prob.n)
    assert np.linalg.norm(X - Xd) <= 1e-8 * np.linalg.norm(Xd)


def test_reciprocity_colocated_C1():
    wl = synthetic.make_workload(synthetic.get_config("C1"))
    assert np.array_equal(wl.src_cells, wl.det_cells)
    prob = problem.build(wl)
    A = prob.operator(wl.theta_ref)
    M = est.measurements(A, prob.n, wl.src_cells, wl.det_cells)
    assert M.shape == (16, 16)
    assert np.linalg.norm(M - M.T) <= 1e-13 * np.linalg.norm(M)
    assert np.all(M > 0)       # positive Green's function of an M-matrix


def test_simultaneous_source_linearity():
    wl = synthetic.make_workload(synthetic.get_config("t2d"))
    prob = problem.build(wl)
    A = prob.operator(wl.theta_ref)
    W = est.sample_matrix(wl.w_signs)
    B = est.simultaneous_rhs(prob.N, wl.src_cells, np.eye(len(wl.src_cells)))
    X_all = solvers.direct_solve(A, B, prob.n)
    X_sim = solvers.direct_solve(A, est.simultaneous_rhs(prob.N, wl.src_cells, W), prob.n)
    assert np.linalg.norm(X_sim - X_all @ W) <= 1e-13 * np.linalg.norm(X_sim)
