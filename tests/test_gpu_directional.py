"""dot_dadp_apply: the derivative of A(p) along parameter directions applied to
fields, Y[:, j] = (sum_k Theta[k, j] dA/dp_k) X[:, j], against the oracle's
definition dA/dp_k = h^d diag(d mu / d p_k) (the columns of G), on grids that
are ragged against the kernel's cell tiles, with more directions than one
pass of the kernel holds; and the matrix-free identity it exists for:
z^T (dA/dp_k) u equals minus the Jacobian entry (eq. Jacobian kth column)."""

import numpy as np
import pytest
import torch

import synthetic
from oracle import problem as oprob

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dl():
    import paper_1706_05586_amd as m
    return m


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


@pytest.mark.parametrize("name,k", [("t2d", 3), ("t3d", 11), ("t3d_c", 17)])
def test_directional_derivative_against_oracle(dl, dev, name, k):
    wl = synthetic.make_workload(synthetic.get_config(name))
    cfg = wl.cfg
    prob = oprob.build(wl)
    G = prob.G(wl.theta_ref)                 # N x n_p
    rng = np.random.default_rng(k)
    Th = rng.standard_normal((cfg.n_p, k))
    X = rng.standard_normal((prob.N, k))
    Y_ref = (G @ Th) * X
    grid, pals = dl.Grid.from_config(cfg), dl.Pals.from_config(cfg)
    th = torch.tensor(wl.theta_ref, device=dev)
    _, D = dl.pals_field(grid, pals, th, cfg.mus_prime)
    with dl.Operator(grid, D) as op:
        op.pals_mua(pals, th)
        Y = op.dadp_apply(torch.tensor(Th, device=dev), torch.tensor(X, device=dev)).cpu().numpy()
        # a unit direction k picks the Jacobian column: -z^T (dA/dp_k) u
        U = rng.standard_normal((prob.N, 1))
        Zf = rng.standard_normal((prob.N, 1))
        Ut, Zt = torch.tensor(U, device=dev), torch.tensor(Zf, device=dev)
        J = op.jacobian(Ut, Zt, dl.DOT_JAC_FP64).cpu().numpy()[0]
        E = torch.eye(cfg.n_p, dtype=torch.float64, device=dev)
        Yk = op.dadp_apply(E, Ut.expand(prob.N, cfg.n_p).contiguous()).cpu().numpy()
    err = np.linalg.norm(Y - Y_ref) / np.linalg.norm(Y_ref)
    print(f"[dA {name}] k={k} rel err {err:.2e}, nonzero rows {np.count_nonzero(Y[:, 0])}",
          flush=True)
    assert err <= 1e-13
    assert np.array_equal(Y == 0, Y_ref == 0) or np.all(np.abs(Y[Y_ref == 0]) == 0)
    mf = -(Zf[:, 0] @ Yk)
    assert np.allclose(mf, J, rtol=1e-12, atol=1e-12 * np.abs(J).max())
