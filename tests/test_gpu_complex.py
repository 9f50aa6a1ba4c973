"""Frequency-domain solves (dot_solve_complex: COCG on (A + i kappa h^d I))
against the oracle's complex direct solve (scipy SuperLU on the same
matrix), on grids with and without a multigrid hierarchy, several
frequencies, forward and adjoint (the matrix is complex symmetric, so the
same call serves both); kappa = 0 reproduces the real solve; the true
relative residual of every column is recomputed on the CPU."""

import numpy as np
import pytest
import torch

import synthetic
from oracle import frequency as ofreq
from oracle import problem as oprob

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dl():
    import paper_1706_05586_amd as m
    return m


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


@pytest.mark.parametrize("name,kappa", [("t3d_b", 0.0), ("t3d_b", 40.0), ("t3d_b", 400.0),
                                        ("t3d_c", 40.0), ("t2d", 40.0), ("inv_t", 40.0)])
def test_complex_solve_matches_direct(dl, dev, name, kappa):
    wl = synthetic.make_workload(synthetic.get_config(name))
    cfg = wl.cfg
    prob = oprob.build(wl)
    Aw = ofreq.operator(prob, wl.theta_ref, kappa)
    rng = np.random.default_rng(7)
    k = 5
    Bc = rng.standard_normal((prob.N, k)) + 1j * rng.standard_normal((prob.N, k))
    Xr = ofreq.direct_solve(Aw, Bc)
    grid, pals = dl.Grid.from_config(cfg), dl.Pals.from_config(cfg)
    th = torch.tensor(wl.theta_ref, device=dev)
    _, D = dl.pals_field(grid, pals, th, cfg.mus_prime)
    with dl.Operator(grid, D) as op:
        op.pals_mua(pals, th)
        for precond in (dl.DOT_PRECOND_AUTO, dl.DOT_PRECOND_JACOBI):
            res = op.solve_complex(torch.tensor(Bc, device=dev), kappa, rtol=1e-12,
                                   precond=precond)
            X = res.x.cpu().numpy()
            rel = ofreq.relative_residuals(Aw, X, Bc)
            fwd = np.linalg.norm(X - Xr, axis=0) / np.linalg.norm(Xr, axis=0)
            print(f"[complex {name} kappa={kappa} precond={precond} levels={op.multigrid_levels}] "
                  f"iters {res.iters_max} relres {rel.max():.2e} (reported {res.relres.max():.2e})"
                  f" forward err {fwd.max():.2e}", flush=True)
            assert res.converged
            assert np.all(rel <= 1.5e-12)
            assert np.allclose(rel, res.relres, rtol=1e-2, atol=1e-15)
            assert fwd.max() <= 1e-8
            if precond == dl.DOT_PRECOND_AUTO:
                fp64_its, fp64_x = res.iters_max, X
            else:
                jac_x = X
        # the binary32 V-cycle (bfloat16 vectors) as preconditioner of the
        # binary64 COCG: the same accuracy; at this tight tolerance the
        # rounded preconditioner costs a few more iterations
        res_m = op.solve_complex(torch.tensor(Bc, device=dev), kappa, rtol=1e-12,
                                 precision=dl.DOT_MIXED)
        Xm = res_m.x.cpu().numpy()
        rel_m = ofreq.relative_residuals(Aw, Xm, Bc)
        print(f"[complex {name} kappa={kappa} mixed V-cycle] iters {res_m.iters_max} "
              f"(binary64 V-cycle {fp64_its}) relres {rel_m.max():.2e}", flush=True)
        assert res_m.converged and np.all(rel_m <= 1.5e-12)
        assert np.linalg.norm(Xm - Xr) <= 1e-8 * np.linalg.norm(Xr)
        if op.multigrid_levels >= 2:
            assert res_m.iters_max <= 1.5 * fp64_its + 2
        else:  # no V-cycle: nothing runs in binary32
            assert np.array_equal(Xm, fp64_x)
        res_j = op.solve_complex(torch.tensor(Bc, device=dev), kappa, rtol=1e-12,
                                 precond=dl.DOT_PRECOND_JACOBI, precision=dl.DOT_MIXED)
        assert np.array_equal(res_j.x.cpu().numpy(), jac_x)
        if kappa == 0.0:
            # the real solve of the same right-hand sides
            Rr = op.solve(torch.tensor(Bc.real, device=dev), rtol=1e-12).x.cpu().numpy()
            assert np.linalg.norm(X.real - Rr) <= 1e-9 * np.linalg.norm(Rr)
