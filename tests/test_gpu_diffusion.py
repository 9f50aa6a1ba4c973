"""Diffusion inverted as well (dot_pals_mua_diffusion): D = 1 / (3 (mu + mu_s))
with both optical properties from the level set, and dA/dp_k with its face
terms (7 diagonals in 3D, 5 in 2D).  Against the oracle (oracle/diffusion.py):
the operator applied to fields, the solves' residuals by the oracle's CSR
matrix, the sampled Jacobian in every precision (also beyond one
contraction tile) and the gradient on the same fields; and the return to the
absorption-only model."""

import numpy as np
import pytest
import torch

import synthetic
from oracle import diffusion as odif
from oracle import estimators as oest
from oracle import problem as oprob
from oracle import solvers as osol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dl():
    import paper_1706_05586_amd as m
    return m


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def _setup(dl, dev, wl, mus_in, mus_out):
    cfg = wl.cfg
    grid, pals = dl.Grid.from_config(cfg), dl.Pals.from_config(cfg)
    th = torch.tensor(wl.theta_ref, device=dev)
    _, D0 = dl.pals_field(grid, pals, th, cfg.mus_prime)
    op = dl.Operator(grid, D0)
    mu, D = op.pals_mua_diffusion(pals, th, mus_in, mus_out)
    return op, pals, th, mu, D


@pytest.mark.parametrize("name", ["t3d", "t2d", "t3d_c"])
def test_operator_solve_jacobian_gradient(dl, dev, name):
    wl = synthetic.make_workload(synthetic.get_config(name))
    cfg = wl.cfg
    prob = oprob.build(wl)
    mus_out = cfg.mus_prime
    mus_in = 2.0 * mus_out
    A = odif.operator(prob, wl.theta_ref, mus_in, mus_out)
    mu_r, D_r, _ = odif.coefficients(prob, wl.theta_ref, mus_in, mus_out)
    W, V = oest.sample_matrix(wl.w_signs), oest.sample_matrix(wl.v_signs)
    ls, ld = W.shape[1], V.shape[1]
    op, pals, th, mu, D = _setup(dl, dev, wl, mus_in, mus_out)
    with op:
        assert np.allclose(D.cpu().numpy(), D_r, rtol=1e-14, atol=0)
        rng = np.random.default_rng(3)
        X = rng.standard_normal((prob.N, 3))
        AX = op.apply(torch.tensor(X, device=dev)).cpu().numpy()
        assert np.linalg.norm(AX - A @ X) <= 1e-13 * np.linalg.norm(A @ X)
        rhs = dl.empty_colmajor(prob.N, ls + ld, dev)
        op.form_rhs(wl.src_cells, torch.tensor(W, device=dev), out=rhs[:, :ls])
        op.form_rhs(wl.det_cells, torch.tensor(V, device=dev), out=rhs[:, ls:])
        res = op.solve(rhs, rtol=1e-12)
        Xs, B = res.x.cpu().numpy(), rhs.cpu().numpy()
        rel = osol.relative_residuals(A, Xs, B)
        assert res.converged and np.all(rel <= 1.5e-12), rel.max()
        U, Z = res.x[:, :ls], res.x[:, ls:]
        Jr = odif.jacobian(prob, wl.theta_ref, mus_in, mus_out, Xs[:, :ls], Xs[:, ls:])
        errs = {}
        for prec, tol in ((dl.DOT_JAC_FP64, 1e-12), (dl.DOT_JAC_SPLIT_BF16X3, 1e-6),
                          (dl.DOT_JAC_SPLIT_BF16, 2e-5)):
            J = op.jacobian(U, Z, prec).cpu().numpy()
            errs[prec] = np.linalg.norm(J - Jr) / np.linalg.norm(Jr)
            assert errs[prec] <= tol, (prec, errs[prec])
        Rs = torch.tensor(rng.standard_normal((ld, ls)), device=dev)
        g = op.grad_misfit(U, Z, Rs).cpu().numpy()
        g_r = Jr.T @ Rs.cpu().numpy().reshape(-1, order="F")
        eg = np.linalg.norm(g - g_r) / np.linalg.norm(g_r)
        # the face terms matter: the absorption-only Jacobian differs
        J_mu = oest.jacobian_sparse_loops(Xs[:, :ls], Xs[:, ls:], prob.G(wl.theta_ref))
        share = np.linalg.norm(Jr - J_mu) / np.linalg.norm(Jr)
        print(f"[diffusion {name}] iters {res.iters_max}, J errors {errs}, gradient {eg:.2e}, "
              f"face-term share of J {share:.2e}", flush=True)
        assert eg <= 1e-12
        assert share > 1e-3
        # back to the absorption-only model: the build-time D again
        op.pals_mua(pals, th)
        A0 = prob.operator(wl.theta_ref)
        AX0 = op.apply(torch.tensor(X, device=dev)).cpu().numpy()
        assert np.linalg.norm(AX0 - A0 @ X) <= 1e-13 * np.linalg.norm(A0 @ X)


@pytest.mark.parametrize("l_s,l_d", [(70, 60), (5, 150)])
def test_tiled_face_contraction(dl, dev, l_s, l_d):
    wl = synthetic.make_workload(synthetic.get_config("t3d"))
    cfg = wl.cfg
    prob = oprob.build(wl)
    mus_out = cfg.mus_prime
    mus_in = 3.0 * mus_out
    rng = np.random.default_rng(l_s + l_d)
    U = rng.standard_normal((prob.N, l_s))
    Z = rng.standard_normal((prob.N, l_d))
    Jr = odif.jacobian(prob, wl.theta_ref, mus_in, mus_out, U, Z)
    op, pals, th, mu, D = _setup(dl, dev, wl, mus_in, mus_out)
    with op:
        Ut = dl.empty_colmajor(prob.N, l_s, dev)
        Ut.copy_(torch.tensor(U, device=dev))
        Zt = dl.empty_colmajor(prob.N, l_d, dev)
        Zt.copy_(torch.tensor(Z, device=dev))
        for prec, tol in ((dl.DOT_JAC_FP64, 1e-12), (dl.DOT_JAC_SPLIT_BF16X3, 1e-6)):
            J = op.jacobian(Ut, Zt, prec).cpu().numpy()
            e = np.linalg.norm(J - Jr) / np.linalg.norm(Jr)
            print(f"[diffusion tiles {l_s}x{l_d}] precision {prec}: {e:.2e}", flush=True)
            assert e <= tol
