"""Pins of the frequency-domain oracle (oracle/frequency.py).

  * constant coefficients with all-Dirichlet faces: A is diagonalized by the
    DST-II, so A + i kappa h^d I is too (eigenvalues lambda + i kappa h^d), and
    scipy's dstn / idstn give the exact complex solution;
  * kappa = 0 reduces to the real oracle (banded Cholesky);
  * A_w is complex symmetric, and the measurements of co-located optodes are
    reciprocal, M = M^T (not M = M^H);
  * the complex sampled Jacobian against central differences of the complex
    sampled residual, and the gradient of f = 1/2 ||r||^2 against central
    differences of f, with the real and imaginary parts stacked.
"""

import numpy as np
import pytest
import scipy.fft as sfft

import synthetic
from oracle import discretization as disc
from oracle import estimators as est
from oracle import frequency as fq
from oracle import problem as oprob
from oracle import solvers


def test_constant_coefficients_match_complex_dst():
    n = (9, 7, 6)
    d = len(n)
    N = int(np.prod(n))
    h = 1.0 / n[0]
    Dc, mu, kappa = 0.31, 0.04, 25.0
    A = disc.assemble(n, (0,) * 6, np.full(N, Dc), np.full(N, mu))

    class P:                       # the two attributes fq.operator reads
        pass
    prob = P()
    prob.h, prob.d, prob.N = h, d, N
    prob.operator = lambda th: A
    Aw = fq.operator(prob, None, kappa)
    shape = disc.cell_shape(n)
    lam = np.zeros(shape)
    for a in range(d):
        k = np.arange(1, n[a] + 1)
        sh = [1] * d
        sh[d - 1 - a] = n[a]
        lam = lam + (2.0 - 2.0 * np.cos(np.pi * k / n[a])).reshape(sh)
    lam = h ** (d - 2) * Dc * lam + h ** d * mu + 1j * kappa * h ** d
    rng = np.random.default_rng(1)
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    bt = sfft.dstn(b.reshape(shape), type=2, norm="ortho")
    x_ref = sfft.idstn(bt / lam, type=2, norm="ortho").ravel()
    x = fq.direct_solve(Aw, b)
    assert np.linalg.norm(x - x_ref) <= 1e-12 * np.linalg.norm(x_ref)


def test_zero_frequency_is_the_real_model():
    wl = synthetic.make_workload(synthetic.get_config("t3d"))
    prob = oprob.build(wl)
    A = prob.operator(wl.theta_ref)
    B = est.simultaneous_rhs(prob.N, wl.src_cells, np.eye(len(wl.src_cells)))
    X = solvers.banded_cholesky_solve(A, B, prob.n)
    Xc = fq.direct_solve(fq.operator(prob, wl.theta_ref, 0.0), B)
    assert np.abs(Xc.imag).max() == 0.0
    assert np.linalg.norm(Xc.real - X) <= 1e-12 * np.linalg.norm(X)


def test_complex_symmetry_and_reciprocity():
    wl = synthetic.make_workload(synthetic.get_config("C1"))
    prob = oprob.build(wl)
    Aw = fq.operator(prob, wl.theta_ref, 30.0)
    assert abs(Aw - Aw.T).max() == 0.0
    assert abs(Aw - Aw.conj().T).max() > 0.0
    M = fq.measurements(prob, wl, wl.theta_ref, 30.0)
    assert np.abs(M.imag).max() > 1e-3 * np.abs(M).max()
    assert np.linalg.norm(M - M.T) <= 1e-12 * np.linalg.norm(M)
    assert np.linalg.norm(M - M.conj().T) > 1e-3 * np.linalg.norm(M)


def test_complex_jacobian_and_gradient_by_central_differences():
    wl = synthetic.make_workload(synthetic.get_config("t3d"))
    cfg = wl.cfg
    prob = oprob.build(wl)
    kappa = 40.0
    rng = np.random.default_rng(2)
    W, V = est.sample_matrix(wl.w_signs), est.sample_matrix(wl.v_signs)
    data = fq.measurements(prob, wl, wl.theta_true, kappa)
    out = fq.evaluate(prob, wl, wl.theta_ref, kappa, W, V, data)
    cols = [(m, a) for m in range(cfg.m0) for a in range(cfg.n_active_per_rbf)]
    # step 1e-5 as for the real Jacobian: smaller steps are dominated by the
    # direct solver's roundoff (cond * eps / h), the truncation is O(h^2)
    h = 1e-5
    scale_J, scale_g = np.abs(out["J"]).max(), np.abs(out["g"]).max()
    for kk in rng.choice(len(cols), size=10, replace=False):
        m, a = cols[kk]
        tp, tm = wl.theta_ref.copy(), wl.theta_ref.copy()
        tp[m, a] += h
        tm[m, a] -= h
        rp = fq.evaluate(prob, wl, tp, kappa, W, V, data)
        rm = fq.evaluate(prob, wl, tm, kappa, W, V, data)
        fd_r = (rp["r"] - rm["r"]) / (2 * h)
        assert np.max(np.abs(fd_r - out["J"][:, kk])) <= 2e-6 * scale_J, kk
        fd_f = (rp["f"] - rm["f"]) / (2 * h)
        assert abs(fd_f - out["g"][kk]) <= 2e-6 * scale_g, kk
    # the imaginary part of the model is not negligible at this frequency
    assert np.abs(out["Jc"].imag).max() > 1e-2 * np.abs(out["Jc"].real).max()
