"""Pins of the oracle's outer inversion driver (oracle/inversion.py).

  * the trust-region truncated-SVD step: with no radius limit and every
    singular value kept it is the minimum-norm least-squares step (numpy
    lstsq) and its model reduction equals 1/2 ||r||^2 - 1/2 ||r + J d||^2
    computed directly; a radius below the first coefficient gives a step of
    exactly that length along the first right singular vector; otherwise the
    kept count is the largest whose step fits;
  * a linear residual r(p) = A p - b: one accepted step reaches the
    least-squares minimum (reduction ratio 1, FE = 2, JE = 1);
  * Rosenbrock's residual (10 (p2 - p1^2), 1 - p1): from (-1.2, 1) the
    phase reaches the minimum (1, 1) with rejected trial steps along the way
    and a monotone accepted misfit;
  * the solve accounting reproduces the totals printed in the paper's tables
    T1 and T3 from their It / FE / JE columns;
  * the full DOT flow on the inversion test grid: the SAA phase and the
    optimized phase lower the sampled misfit monotonically, the true misfit
    falls as well, every solve is counted as the formula says, the optimized
    directions are orthonormal and their complement is orthogonal to them.
"""

import os

import numpy as np
import pytest

import synthetic
from oracle import estimators as oest
from oracle import inversion as inv
from oracle import problem as oprob

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "solve_counts_T1_T3.txt")


def test_step_is_least_squares_without_a_radius():
    rng = np.random.default_rng(1)
    for rows, cols in ((12, 7), (6, 9)):
        J = rng.standard_normal((rows, cols))
        r = rng.standard_normal(rows)
        Lm, s, Rt = np.linalg.svd(J, full_matrices=False)
        c = Lm.T @ r
        t, kappa, norm, pred = inv.truncated_step_coefficients(s, c, np.inf, 0.0)
        assert t == min(rows, cols) and kappa == 0.0
        d = -(Rt[:t].T @ (c[:t] / s[:t]))
        d_ls = -np.linalg.lstsq(J, r, rcond=None)[0]
        assert np.allclose(d, d_ls, rtol=1e-12, atol=1e-12)
        assert norm == pytest.approx(np.linalg.norm(d_ls), rel=1e-12)
        direct = 0.5 * r @ r - 0.5 * np.sum((r + J @ d) ** 2)
        assert pred == pytest.approx(direct, rel=1e-12)


def test_step_inside_a_radius():
    s = np.array([4.0, 2.0, 1.0, 1e-9])
    c = np.array([2.0, -2.0, 3.0, 5.0])
    # a = c / s = 0.5, -1, 3 (the last singular value is dropped); the
    # leading partial steps have lengths 0.5, sqrt(1.25), sqrt(10.25)
    t, kappa, norm, pred = inv.truncated_step_coefficients(s, c, 1.2, 1e-4)
    k = np.sqrt(1.44 - 1.25) / 3.0
    assert t == 2 and kappa == pytest.approx(k, rel=1e-14) and norm == pytest.approx(1.2)
    assert pred == pytest.approx(0.5 * (4 + 4) + (k - k * k / 2) * 9.0, rel=1e-14)
    t, kappa, norm, pred = inv.truncated_step_coefficients(s, c, 0.2, 1e-4)
    assert t == 0 and kappa == pytest.approx(0.4) and norm == pytest.approx(0.2)
    assert pred == pytest.approx((0.4 - 0.08) * 4.0, rel=1e-14)
    # the tiny singular value is never used, however large the radius
    t, kappa, norm, pred = inv.truncated_step_coefficients(s, c, 1e9, 1e-4)
    assert (t, kappa) == (3, 0.0) and norm == pytest.approx(np.sqrt(10.25))
    # the model reduction of the shortened step, evaluated directly
    J = np.diag(s[:3])
    r = c[:3]
    for radius in (0.2, 0.7, 1.2, 2.0):
        t, kappa, norm, pred = inv.truncated_step_coefficients(s[:3], r, radius, 0.0)
        a = r / s[:3]
        d = -a * np.array([1.0 if i < t else (kappa if i == t else 0.0) for i in range(3)])
        assert np.linalg.norm(d) == pytest.approx(min(radius, np.sqrt(10.25)), rel=1e-13)
        assert pred == pytest.approx(0.5 * r @ r - 0.5 * np.sum((r + J @ d) ** 2), rel=1e-13)


def test_linear_residual_one_step():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((15, 6))
    b = rng.standard_normal(15)

    def evaluate(p):
        r = A @ p - b
        return 0.5 * r @ r, r, None

    opts = inv.TrustRegionOptions(radius0=1e6, rcut=0.0)
    res = inv.tr_gauss_newton(evaluate, lambda p, st: A, np.zeros(6), 0.0, opts)
    p_ls = np.linalg.lstsq(A, b, rcond=None)[0]
    h = res.history[0]
    assert h["accept"] and h["ratio"] == pytest.approx(1.0, rel=1e-10)
    assert np.allclose(res.history[0]["f_trial"], 0.5 * np.sum((A @ p_ls - b) ** 2), rtol=1e-12)
    # a second step from the minimum has no model reduction left
    assert (res.fe, res.je) == (res.it + 1, 2) and res.it <= 2
    assert np.allclose(res.p, p_ls, rtol=1e-10, atol=1e-12)


def test_rosenbrock_residual():
    def evaluate(p):
        r = np.array([10.0 * (p[1] - p[0] ** 2), 1.0 - p[0]])
        return 0.5 * r @ r, r, None

    def jac(p, st):
        return np.array([[-20.0 * p[0], 10.0], [-1.0, 0.0]])

    opts = inv.TrustRegionOptions(radius0=5.0, rcut=1e-12, max_iter=100)
    res = inv.tr_gauss_newton(evaluate, jac, np.array([-1.2, 1.0]), 1e-20, opts)
    assert res.converged and np.allclose(res.p, [1.0, 1.0], atol=1e-9)
    acc = [h for h in res.history if h["accept"]]
    assert any(not h["accept"] for h in res.history)          # the radius did its job
    fs = [h["f_trial"] for h in acc]
    assert all(b < a for a, b in zip(fs, fs[1:]))
    assert res.fe == res.it + 1 and res.je == len(acc)         # no J at the converged point


def test_solve_accounting_reproduces_the_tables():
    class Ph:
        def __init__(self, fe, je):
            self.fe, self.je = fe, je

    rows = 0
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        tab, name, l, n_s, n_d, it, fe, je, total, sfe, sje, upd = line.split()
        l, n_s, n_d, it, fe, je, total, sfe, sje, upd = map(
            int, (l, n_s, n_d, it, fe, je, total, sfe, sje, upd))
        phases = ([Ph(sfe, sje)] if upd else []) + [Ph(fe, je)]
        assert inv.solve_count(phases, l, l, upd, n_s, n_d) == total, (tab, name)
        if tab == "T1":
            assert fe == it + 1, name
        rows += 1
    assert rows == 8


@pytest.mark.slow
def test_dot_flow_on_a_small_grid():
    wl = synthetic.make_workload(synthetic.get_config("inv_t"))
    cfg = wl.cfg
    prob = oprob.build(wl)
    data = oprob.synthetic_data(prob, wl)
    sdot = inv.SampledDOT(prob, wl, data, wl.theta_ref)
    p0 = inv.params_of(wl.theta_ref, prob.active)
    W0, V0 = oest.sample_matrix(wl.w_signs), oest.sample_matrix(wl.v_signs)
    opts = inv.TrustRegionOptions(radius0=0.5, max_iter=4)
    out = inv.invert(sdot, p0, W0, V0, cfg.q_s, cfg.q_d, wl.y_signs, wl.z_signs, cfg.noise, opts)
    saa, opt = out["saa"], out["opt"]
    for ph in (saa, opt):
        assert ph.fe == ph.it + 1
        fs = [ph.history[0]["f"]] + [h["f_trial"] for h in ph.history if h["accept"]]
        assert all(b < a for a, b in zip(fs, fs[1:]))
    assert out["counted"] == out["solves"] == inv.solve_count(
        [saa, opt], cfg.l_s, cfg.l_d, 1, cfg.n_s, cfg.n_d)
    W, V, q = out["W"], out["V"], cfg.q_s
    assert np.allclose(W[:, :q].T @ W[:, :q], np.eye(q), atol=1e-12)
    assert np.allclose(W[:, :q].T @ W[:, q:], 0.0, atol=1e-12)
    assert np.allclose(V[:, :cfg.q_d].T @ V[:, cfg.q_d:], 0.0, atol=1e-12)
    assert out["J_full"].shape == (cfg.n_s * cfg.n_d, cfg.n_p)
    assert sdot.true_misfit(out["p"]) < 0.5 * sdot.true_misfit(p0)
