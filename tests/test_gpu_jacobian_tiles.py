"""The contraction beyond one pass of the matrix-core kernels: samples whose
source x detector block exceeds what a kernel holds run tile by tile (at
most 64 sources and as many detectors as fit), each tile written into its
rows of J_s (row j + l_d i, detector fastest).  Checked against the oracle's
sparse loop nest on the same fields, with ragged last tiles in both
directions, for every precision; and the full Jacobian of eq. Jtensor
(every source, every detector) on solved fields against the oracle's, whose
fields come from its direct solver."""

import numpy as np
import pytest
import torch

import synthetic
from oracle import estimators as oest
from oracle import problem as oprob

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dl():
    import paper_1706_05586_amd as m
    return m


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def _operator(dl, dev, wl):
    cfg = wl.cfg
    grid, pals = dl.Grid.from_config(cfg), dl.Pals.from_config(cfg)
    _, D = dl.pals_field(grid, pals, torch.tensor(wl.theta_ref, device=dev), cfg.mus_prime)
    op = dl.Operator(grid, D)
    op.pals_mua(pals, torch.tensor(wl.theta_ref, device=dev))
    return op


@pytest.mark.parametrize("l_s,l_d", [(70, 60), (130, 9), (5, 150)])
def test_tiled_jacobian_against_oracle_loops(dl, dev, l_s, l_d):
    wl = synthetic.make_workload(synthetic.get_config("t3d"))
    prob = oprob.build(wl)
    G = prob.G(wl.theta_ref)
    rng = np.random.default_rng(l_s * 1000 + l_d)
    U = rng.standard_normal((prob.N, l_s))
    Z = rng.standard_normal((prob.N, l_d))
    Jr = oest.jacobian_sparse_loops(U, Z, G)
    with _operator(dl, dev, wl) as op:
        Ut = dl.empty_colmajor(prob.N, l_s, dev)
        Ut.copy_(torch.tensor(U, device=dev))
        Zt = dl.empty_colmajor(prob.N, l_d, dev)
        Zt.copy_(torch.tensor(Z, device=dev))
        for prec, tol in ((dl.DOT_JAC_FP64, 1e-13), (dl.DOT_JAC_SPLIT_BF16X3, 1e-6),
                          (dl.DOT_JAC_SPLIT_BF16, 2e-5)):
            J = op.jacobian(Ut, Zt, prec).cpu().numpy()
            e = np.linalg.norm(J - Jr) / np.linalg.norm(Jr)
            rows = np.linalg.norm(J - Jr, axis=1) / np.maximum(np.linalg.norm(Jr, axis=1), 1e-300)
            print(f"[tiles {l_s}x{l_d}] precision {prec}: rel err {e:.2e}, worst row {rows.max():.2e}",
                  flush=True)
            assert e <= tol
            assert rows.max() <= 1e-3        # every tile landed on its own rows


def test_full_jacobian_every_source_and_detector(dl, dev):
    """The full J of eq. Jtensor on the inversion test grid (36 sources,
    36 detectors, 27 RBFs with five parameters): n_s + n_d solves, then
    one contraction (36 x 36 with five parameters per RBF: two detector
    tiles in binary64)."""
    # as a 20 mm slab: the detector readings are then about 3e-5 of the
    # fields' size, so CG fields to relres 1e-12 match the direct solve's
    # J to about 1e-10 (in the 60 mm slab only to about 1e-7)
    L = 20.0
    wl = synthetic.make_workload(synthetic.get_config("inv_t", mu_out=0.01 * L, mu_in=0.05 * L,
                                                      mus_prime=L))
    cfg = wl.cfg
    prob = oprob.build(wl)
    ns, nd = cfg.n_s, cfg.n_d
    ref = oprob.evaluate(prob, wl, wl.theta_ref, np.eye(ns), np.eye(nd), np.zeros((nd, ns)))
    with _operator(dl, dev, wl) as op:
        B = op.form_rhs(wl.src_cells, torch.eye(ns, dtype=torch.float64, device=dev))
        C = op.form_rhs(wl.det_cells, torch.eye(nd, dtype=torch.float64, device=dev))
        U = op.solve(B, rtol=1e-12).x
        Z = op.solve(C, rtol=1e-12, trans=1).x
        J = op.jacobian(U, Z, dl.DOT_JAC_FP64).cpu().numpy()
        J3 = op.jacobian(U, Z, dl.DOT_JAC_SPLIT_BF16X3).cpu().numpy()
        Jl = oest.jacobian_sparse_loops(U.cpu().numpy(), Z.cpu().numpy(), ref["G"])
    assert J.shape == (ns * nd, cfg.n_p) == ref["Js"].shape
    e_same = np.linalg.norm(J - Jl) / np.linalg.norm(Jl)
    e_dir = np.linalg.norm(J - ref["Js"]) / np.linalg.norm(ref["Js"])
    e3 = np.linalg.norm(J3 - Jl) / np.linalg.norm(Jl)
    print(f"[full J {ns * nd}x{cfg.n_p}] vs loops on the same fields {e_same:.2e}, "
          f"vs the direct-solve J {e_dir:.2e}, 3-part split {e3:.2e}", flush=True)
    assert e_same <= 1e-12
    assert e_dir <= 1e-8
    assert e3 <= 1e-6
