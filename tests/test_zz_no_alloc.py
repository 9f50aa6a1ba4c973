"""The allocation-free gradient entry point (dot_grad_misfit_noalloc) against
dot_grad_misfit, which takes the caller's workspace: both run the same
kernels in the same order, so the gradients must agree bit for bit.  Three
calls in a row share the library's fixed scratch array: a 24^3 grid, then a
smaller 19 x 13 x 11 grid, then that grid with 40 source fields (the other
per-cell kernel); stale values left by a larger call must not leak into a
smaller one.  A grid whose scratch exceeds the fixed array is rejected."""

import numpy as np
import pytest
import torch

import synthetic
from oracle import estimators as oest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dl():
    import paper_1706_05586_amd as m
    return m


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def _operator(dl, dev, wl, n=None):
    cfg = wl.cfg
    grid = dl.Grid.from_config(cfg) if n is None else dl.Grid(dim=3, n=n, bc=tuple(cfg.bc[:6]))
    pals = dl.Pals.from_config(cfg)
    _, D = dl.pals_field(grid, pals, torch.tensor(wl.theta_ref, device=dev), cfg.mus_prime)
    op = dl.Operator(grid, D)
    op.pals_mua(pals, torch.tensor(wl.theta_ref, device=dev))
    return op


def _solved_fields(dl, dev, name):
    wl = synthetic.make_workload(synthetic.get_config(name))
    op = _operator(dl, dev, wl)
    W = torch.tensor(oest.sample_matrix(wl.w_signs), device=dev)
    V = torch.tensor(oest.sample_matrix(wl.v_signs), device=dev)
    ls, ld = W.shape[1], V.shape[1]
    rhs = dl.empty_colmajor(op.N, ls + ld, dev)
    op.form_rhs(wl.src_cells, W, out=rhs[:, :ls])
    op.form_rhs(wl.det_cells, V, out=rhs[:, ls:])
    x = op.solve(rhs, rtol=1e-12).x
    return op, x[:, :ls], x[:, ls:]


def _random_colmajor(dl, dev, rng, rows, cols):
    t = dl.empty_colmajor(rows, cols, dev)
    t.copy_(torch.tensor(rng.standard_normal((rows, cols)), device=dev))
    return t


def test_noalloc_gradient_matches_workspace_gradient(dl, dev):
    rng = np.random.default_rng(2024)
    cases = [("t3d_b", None), ("t3d", None), ("t3d", 40)]
    for name, l_s in cases:
        op, U, Z = _solved_fields(dl, dev, name)
        with op:
            if l_s is not None:          # random fields with more source columns
                U = _random_colmajor(dl, dev, rng, op.N, l_s)
            ls, ld = U.shape[1], Z.shape[1]
            Rs = _random_colmajor(dl, dev, rng, ld, ls)
            g_ref = op.grad_misfit(U, Z, Rs)
            out = torch.full_like(g_ref, float("nan"))
            g = op.grad_misfit_noalloc(U, Z, Rs, out)
            torch.cuda.synchronize()
            print(f"[noalloc] {name} N={op.N} l_s={ls} l_d={ld} n_p={g.numel()} "
                  f"|g|={torch.linalg.norm(g_ref).item():.3e}", flush=True)
            assert torch.linalg.norm(g_ref).item() > 0
            assert torch.equal(g, g_ref)


def test_noalloc_gradient_rejects_grids_beyond_the_scratch(dl, dev):
    wl = synthetic.make_workload(synthetic.get_config("t3d"))
    n = (256, 128, 128)                  # 2^22 cells: no room for the chunk partials
    op = _operator(dl, dev, wl, n=n)
    with op:
        U = dl.empty_colmajor(op.N, 1, dev)
        Z = dl.empty_colmajor(op.N, 1, dev)
        U.zero_()
        Z.zero_()
        Rs = torch.zeros((1, 1), dtype=torch.float64, device=dev)
        n_p = op.pals.m0 * op.pals.n_act(3)
        out = torch.zeros(n_p, dtype=torch.float64, device=dev)
        with pytest.raises(dl.DotError) as ei:
            op.grad_misfit_noalloc(U, Z, Rs, out)
        assert ei.value.code == dl._lib.DOT_EINVAL
        assert "fixed gradient scratch" in str(ei.value)
        # the workspace entry point still serves this grid
        g = op.grad_misfit(U, Z, Rs)
        torch.cuda.synchronize()
        assert torch.count_nonzero(g).item() == 0
