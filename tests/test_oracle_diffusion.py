"""Pins of the diffusion-inverting oracle (oracle/diffusion.py).

  * dA/dp_k by the chain rule against central differences of the assembled
    A(p) (every entry, O(h^2) agreement), symmetric, with off-diagonal
    entries (7 diagonals in 3D, 5 in 2D);
  * when the scattering contrast cancels the absorption contrast
    (mus_in - mus_out = -(mu_in - mu_out)), D is constant and dA/dp_k reduces
    to the diagonal h^d d mu / d p_k of the absorption-only model;
  * the sampled Jacobian against central differences of the sampled residual
    (the real and the 2D grid).
"""

import numpy as np
import pytest

import synthetic
from oracle import diffusion as dif
from oracle import estimators as est
from oracle import pals
from oracle import problem as oprob
from oracle import solvers


def _params(wl, prob):
    return pals.params_from_theta(wl.theta_ref, prob.active)


@pytest.mark.parametrize("name", ["t3d", "t2d"])
def test_dA_dp_matches_central_differences(name):
    wl = synthetic.make_workload(synthetic.get_config(name))
    prob = oprob.build(wl)
    mus_in, mus_out = 2.0, 1.0
    D, dmu, dD = dif.derivative_fields(prob, wl.theta_ref, mus_in, mus_out)
    p0 = _params(wl, prob)
    h = 1e-6
    rng = np.random.default_rng(0)
    nz = [k for k in range(p0.size) if np.any(dmu[:, k])]
    for k in rng.choice(nz, size=min(6, len(nz)), replace=False):
        Mk = dif.dA_dp(prob, D, dD[:, k], dmu[:, k])
        assert abs(Mk - Mk.T).max() == 0.0
        pp, pm = p0.copy(), p0.copy()
        pp[k] += h
        pm[k] -= h
        Ap = dif.operator(prob, pals.theta_from_params(wl.theta_ref, pp, prob.active), mus_in, mus_out)
        Am = dif.operator(prob, pals.theta_from_params(wl.theta_ref, pm, prob.active), mus_in, mus_out)
        fd = (Ap - Am) / (2 * h)
        err = abs(fd - Mk).max()
        assert err <= 1e-6 * abs(Mk).max(), (k, err)
        off = Mk - Mk.multiply(np.eye(Mk.shape[0], dtype=bool))
        assert abs(off).max() > 0.0        # the diffusion part is there


def test_cancelling_contrasts_reduce_to_the_absorption_model():
    wl = synthetic.make_workload(synthetic.get_config("t3d"))
    prob = oprob.build(wl)
    c = prob.consts
    mus_out = 1.0
    mus_in = mus_out - (c["mu_in"] - c["mu_out"])
    D, dmu, dD = dif.derivative_fields(prob, wl.theta_ref, mus_in, mus_out)
    # the two contrasts cancel up to the rounding of their ratio
    assert np.ptp(D) <= 1e-15 * D.max() and np.abs(dD).max() <= 1e-14 * np.abs(dmu).max()
    for k in range(0, dmu.shape[1], 7):
        Mk = dif.dA_dp(prob, D, dD[:, k], dmu[:, k])
        ref = np.diag(prob.h ** 3 * dmu[:, k])
        assert abs(Mk - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300)


@pytest.mark.parametrize("name", ["t3d", "t2d"])
def test_jacobian_matches_central_differences_of_the_residual(name):
    wl = synthetic.make_workload(synthetic.get_config(name))
    prob = oprob.build(wl)
    mus_in, mus_out = 2.0, 1.0
    W, V = est.sample_matrix(wl.w_signs), est.sample_matrix(wl.v_signs)
    p0 = _params(wl, prob)

    def fields(p):
        A = dif.operator(prob, pals.theta_from_params(wl.theta_ref, p, prob.active), mus_in, mus_out)
        U = solvers.direct_solve(A, est.simultaneous_rhs(prob.N, wl.src_cells, W), prob.n)
        Z = solvers.direct_solve(A, est.simultaneous_rhs(prob.N, wl.det_cells, V), prob.n)
        return U, Z

    U, Z = fields(p0)
    J = dif.jacobian(prob, wl.theta_ref, mus_in, mus_out, U, Z)

    def resid(p):
        U, _ = fields(p)
        return (V.T @ U[wl.det_cells, :]).reshape(-1, order="F")

    hstep = 1e-5
    scale = np.abs(J).max()
    for k in range(p0.size):
        pp, pm = p0.copy(), p0.copy()
        pp[k] += hstep
        pm[k] -= hstep
        fd = (resid(pp) - resid(pm)) / (2 * hstep)
        assert np.max(np.abs(fd - J[:, k])) <= 2e-6 * scale, k
