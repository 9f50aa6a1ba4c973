"""Pins for the oracle's randomized estimators (Section 3.1).

* with W = I, V = I the sampled misfit is exactly 1/2 ||R||_F^2;
* Thm. 3.1 (E ||V^T R W||_F^2 = ||R||_F^2) by exact enumeration of every
  Rademacher sign pattern on a small problem;
* unbiased gradient and Gauss-Newton Hessian (eqs. UnbiasedGrad/UnbiasedHess)
  by exact enumeration;
* Kronecker identity J_s = (W^T kron V^T) J on real PDE fields, J computed
  from all sources/detectors, J_s from simultaneous ones;
* the loop-nest Jacobian against central finite differences of the residual;
* the gradient by two routes, and against central differences of the misfit.
"""

import itertools

import numpy as np
import pytest

import synthetic
from oracle import estimators as est
from oracle import pals, problem, solvers


def _all_sign_matrices(rows, cols):
    for bits in itertools.product((-1, 1), repeat=rows * cols):
        yield np.array(bits, dtype=np.int8).reshape(rows, cols)


def test_full_sample_gives_true_misfit():
    rng = np.random.default_rng(1)
    n_d, n_s = 5, 4
    M, Dd = rng.standard_normal((n_d, n_s)), rng.standard_normal((n_d, n_s))
    det = np.arange(n_d)
    W, V = np.eye(n_s), np.eye(n_d)
    Rs = est.sampled_residual(M @ W, det, V, Dd @ W)
    assert 2 * est.misfit(Rs) == pytest.approx(np.sum((M - Dd) ** 2), rel=1e-15)


@pytest.mark.parametrize("ls,ld", [(1, 1), (2, 1), (1, 2)])
def test_theorem_3_1_exact_enumeration(ls, ld):
    rng = np.random.default_rng(2)
    n_d, n_s = 3, 3
    M, Dd = rng.standard_normal((n_d, n_s)), rng.standard_normal((n_d, n_s))
    det = np.arange(n_d)
    vals = []
    for ws in _all_sign_matrices(n_s, ls):
        W = est.sample_matrix(ws)
        for vs in _all_sign_matrices(n_d, ld):
            V = est.sample_matrix(vs)
            vals.append(2 * est.misfit(est.sampled_residual(M @ W, det, V, Dd @ W)))
    assert np.mean(vals) == pytest.approx(np.sum((M - Dd) ** 2), rel=1e-13)
    assert np.var(vals) > 0   # a genuine estimator, not an identity


def test_unbiased_gradient_and_hessian_exact_enumeration():
    rng = np.random.default_rng(3)
    n_d, n_s, n_p = 3, 2, 4
    J = rng.standard_normal((n_d * n_s, n_p))
    r = rng.standard_normal(n_d * n_s)
    g_sum = np.zeros(n_p)
    H_sum = np.zeros((n_p, n_p))
    count = 0
    for ws in _all_sign_matrices(n_s, 1):
        W = est.sample_matrix(ws)
        for vs in _all_sign_matrices(n_d, 1):
            V = est.sample_matrix(vs)
            S = np.kron(W, V).T
            Js, rs = S @ J, S @ r
            g_sum += Js.T @ rs
            H_sum += Js.T @ Js
            count += 1
    assert np.allclose(g_sum / count, J.T @ r, atol=1e-13)
    assert np.allclose(H_sum / count, J.T @ J, atol=1e-13)


def _fields(prob, wl, A, W, V):
    BW = est.simultaneous_rhs(prob.N, wl.src_cells, W)
    CV = est.simultaneous_rhs(prob.N, wl.det_cells, V)
    return solvers.direct_solve(A, BW, prob.n), solvers.direct_solve(A, CV, prob.n)


@pytest.mark.parametrize("name", ["t2d", "t3d"])
def test_kronecker_identity_on_pde_fields(name):
    wl = synthetic.make_workload(synthetic.get_config(name))
    prob = problem.build(wl)
    theta = wl.theta_ref
    A = prob.operator(theta)
    G = prob.G(theta)
    n_s, n_d = len(wl.src_cells), len(wl.det_cells)
    U_all, Z_all = _fields(prob, wl, A, np.eye(n_s), np.eye(n_d))
    J_full = est.jacobian_loops(U_all, Z_all, G)
    W, V = est.sample_matrix(wl.w_signs), est.sample_matrix(wl.v_signs)
    U, Z = _fields(prob, wl, A, W, V)
    Js = est.jacobian_loops(U, Z, G)
    assert np.abs(G).max() > 0
    ref = np.kron(W, V).T @ J_full
    assert np.linalg.norm(Js - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.allclose(est.jacobian_sparse_loops(U, Z, G), Js, rtol=0, atol=1e-14 * np.abs(Js).max())


@pytest.mark.parametrize("name", ["t2d", "t3d"])
def test_jacobian_matches_central_fd_of_residual(name):
    wl = synthetic.make_workload(synthetic.get_config(name))
    prob = problem.build(wl)
    theta = wl.theta_ref
    active = wl.cfg.active
    n_s, n_d = len(wl.src_cells), len(wl.det_cells)
    A = prob.operator(theta)
    U_all, Z_all = _fields(prob, wl, A, np.eye(n_s), np.eye(n_d))
    J = est.jacobian_loops(U_all, Z_all, prob.G(theta))
    p0 = pals.params_from_theta(theta, active)

    def resid(p):
        Ap = prob.operator(pals.theta_from_params(theta, p, active))
        return est.measurements(Ap, prob.n, wl.src_cells, wl.det_cells).reshape(-1, order="F")

    # step 1e-5: smaller steps are dominated by the direct solver's roundoff
    # (kappa * eps / h); the truncation error is O(h^2) ~ 1e-10 relative
    hstep = 1e-5
    for k in range(p0.size):
        pp, pm = p0.copy(), p0.copy()
        pp[k] += hstep
        pm[k] -= hstep
        fd = (resid(pp) - resid(pm)) / (2 * hstep)
        scale = np.abs(J).max()
        assert np.max(np.abs(fd - J[:, k])) <= 2e-6 * scale, k


def test_gradient_two_routes_and_fd():
    wl = synthetic.make_workload(synthetic.get_config("t3d"))
    prob = problem.build(wl)
    data = problem.synthetic_data(prob, wl)
    W, V = est.sample_matrix(wl.w_signs), est.sample_matrix(wl.v_signs)
    theta = wl.theta_ref
    out = problem.evaluate(prob, wl, theta, W, V, data)
    g1 = est.gradient_via_jacobian(out["Js"], out["Rs"])
    g2 = out["g"]
    assert np.linalg.norm(g1 - g2) <= 1e-12 * np.linalg.norm(g1)
    active = wl.cfg.active
    p0 = pals.params_from_theta(theta, active)

    def f(p):
        th = pals.theta_from_params(theta, p, active)
        return problem.evaluate(prob, wl, th, W, V, data, with_jacobian=False)["f"]

    hstep = 1e-5
    fd = np.empty(p0.size)
    for k in range(p0.size):
        pp, pm = p0.copy(), p0.copy()
        pp[k] += hstep
        pm[k] -= hstep
        fd[k] = (f(pp) - f(pm)) / (2 * hstep)
    assert np.max(np.abs(fd - g1)) <= 2e-6 * np.abs(g1).max()
