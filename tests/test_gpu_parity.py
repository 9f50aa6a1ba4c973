"""GPU parity: every ABI call against the CPU oracle on the same seeded inputs.

Grids are ragged against the kernels' 64 x 8 tiles and z chunks (37x29,
19x13x11, 24^3, 70x33x17, 32^2).  Tolerances:
  * PaLS mu and D, stencil apply: 1e-13 relative (binary64 rounding only);
  * RHS scatter: exact;
  * FP64 solve: true relative residual, recomputed by the oracle's CSR
    matrix, at most the requested rtol (1e-12) times 1.5 (the final true
    residual is not the recursive one); with Jacobi preconditioning the
    iteration counts within 3% of the oracle's Jacobi-PCG, with the
    multigrid V-cycle (grids that halve: 24^3) fewer than half of them;
    bitwise reproducible;
  * mixed solve: true relative residual <= rtol;
  * one V-cycle (dot_multigrid_apply) against the scipy model of the same
    preconditioner (tests/mg_reference.py): 1e-12;
  * misfit, Jacobian (given identical fields), gradient: 1e-12 relative.
"""

import numpy as np
import pytest
import torch

import synthetic
from oracle import discretization as odisc
from oracle import estimators as oest
from oracle import problem as oprob
from oracle import solvers as osol

pytestmark = pytest.mark.gpu

NAMES = ["t2d", "t3d", "t3d_b", "t3d_c", "C1"]


@pytest.fixture(scope="module")
def dotlib():
    import paper_1706_05586_amd as dl
    assert torch.cuda.is_available()
    return dl


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


_CACHE = {}


def case(name):
    if name in _CACHE:
        return _CACHE[name]
    wl = synthetic.make_workload(synthetic.get_config(name))
    prob = oprob.build(wl)
    if name == "C1":   # the 2D workload uses every source and detector (W = V = I)
        W, V = np.eye(len(wl.src_cells)), np.eye(len(wl.det_cells))
    else:
        W, V = oest.sample_matrix(wl.w_signs), oest.sample_matrix(wl.v_signs)
    data = oprob.synthetic_data(prob, wl)
    ref = oprob.evaluate(prob, wl, wl.theta_ref, W, V, data)
    _CACHE[name] = (wl, prob, W, V, data, ref)
    return _CACHE[name]


def gpu_operator(dl, dev, wl, D=None):
    cfg = wl.cfg
    grid, pals = dl.Grid.from_config(cfg), dl.Pals.from_config(cfg)
    th = torch.tensor(wl.theta_ref, device=dev)
    if D is None:
        _, D = dl.pals_field(grid, pals, th, cfg.mus_prime)
    op = dl.Operator(grid, D)
    return op, grid, pals, th


@pytest.mark.parametrize("name", NAMES)
def test_pals_field_matches_oracle(dotlib, dev, name):
    wl, prob, *_ = case(name)
    cfg = wl.cfg
    grid, pals = dotlib.Grid.from_config(cfg), dotlib.Pals.from_config(cfg)
    mua, D = dotlib.pals_field(grid, pals, torch.tensor(wl.theta_ref, device=dev), cfg.mus_prime)
    mu_ref = prob.mua(wl.theta_ref)
    assert np.max(np.abs(mua.cpu().numpy() - mu_ref)) <= 1e-13 * np.max(mu_ref)
    assert np.max(np.abs(D.cpu().numpy() - prob.D)) <= 1e-13 * np.max(prob.D)
    # the workload really has an anomaly band
    assert mu_ref.max() > cfg.mu_out * 1.5 or name == "t3d_c"


@pytest.mark.parametrize("name", NAMES)
def test_apply_matches_oracle_csr(dotlib, dev, name):
    wl, prob, *_ = case(name)
    Dt = torch.tensor(prob.D, device=dev)
    op, grid, pals, th = gpu_operator(dotlib, dev, wl, D=Dt)
    with op:
        rng = np.random.default_rng(7)
        X = rng.standard_normal((prob.N, 5))
        # explicit mu
        mu = prob.mua(wl.theta_ref)
        op.set_mua(torch.tensor(mu, device=dev))
        Y = op.apply(torch.tensor(X, device=dev)).cpu().numpy()
        A = odisc.assemble(prob.n, prob.bc, prob.D, mu)
        Yr = A @ X
        assert np.linalg.norm(Y - Yr) <= 1e-13 * np.linalg.norm(Yr)
        # PaLS-driven mu at theta_ref
        op.pals_mua(pals, th)
        Y2 = op.apply(torch.tensor(X, device=dev)).cpu().numpy()
        assert np.linalg.norm(Y2 - Yr) <= 1e-13 * np.linalg.norm(Yr)


@pytest.mark.parametrize("name", ["t3d", "t2d"])
def test_form_rhs_exact(dotlib, dev, name):
    wl, prob, W, V, data, ref = case(name)
    op, *_ = gpu_operator(dotlib, dev, wl)
    with op:
        BW = op.form_rhs(wl.src_cells, torch.tensor(W, device=dev)).cpu().numpy()
        assert np.array_equal(BW, ref["BW"])
        # repeated cells add up
        cells = np.array([3, 3, 5], dtype=np.int32)
        w = np.array([[1.0, 2.0], [0.5, -1.0], [4.0, 0.0]])
        R = op.form_rhs(cells, torch.tensor(w, device=dev)).cpu().numpy()
        assert R[3, 0] == 1.5 and R[3, 1] == 1.0 and R[5, 0] == 4.0 and np.count_nonzero(R) == 3
        # in the order given: 1 is lost to 1e16 before -1e16 cancels it
        cells = np.array([7, 2, 7, 7], dtype=np.int32)
        w = np.array([[1e16], [2.0], [1.0], [-1e16]])
        R = op.form_rhs(cells, torch.tensor(w, device=dev)).cpu().numpy()
        assert R[7, 0] == 0.0 and R[2, 0] == 2.0 and np.count_nonzero(R) == 1
        # lists seen before, new ones and ones pushed out of the handle's
        # device copies all give the sequential sum
        rng = np.random.default_rng(3)
        lists = [rng.integers(0, op.N, size=n).astype(np.int32) for n in (5, 9, 5, 12, 7, 3)]
        lists.append(lists[0][[0, 0, 1, 2, 0]])
        for _ in range(2):
            for c in lists + lists[:2]:
                w = rng.standard_normal((len(c), 3))
                R = op.form_rhs(c, torch.tensor(w, device=dev)).cpu().numpy()
                E = np.zeros((op.N, 3))
                for i, cell in enumerate(c):
                    E[cell] += w[i]
                assert np.array_equal(R, E)


@pytest.mark.parametrize("precond", ["auto", "jacobi"])
@pytest.mark.parametrize("name", NAMES)
def test_solve_fp64_matches_oracle(dotlib, dev, name, precond):
    wl, prob, W, V, data, ref = case(name)
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    pc = dotlib.DOT_PRECOND_AUTO if precond == "auto" else dotlib.DOT_PRECOND_JACOBI
    with op:
        op.pals_mua(pals, th)
        levels = op.multigrid_levels
        rhs = np.hstack([ref["BW"], ref["CV"]])
        res = op.solve(torch.tensor(rhs, device=dev), rtol=1e-12, precision=dotlib.DOT_FP64,
                       precond=pc)
        X = res.x.cpu().numpy()
    import mg_reference as omg
    # every test grid coarsens: odd sides end in a ragged aggregate, 2D in 2 x 2
    assert levels == len(omg.level_shapes(prob.n))
    assert res.converged
    true_rel = osol.relative_residuals(ref["A"], X, rhs)
    assert np.all(true_rel <= 1.5e-12), true_rel.max()
    assert np.allclose(true_rel, res.relres, rtol=1e-3, atol=1e-15)
    Xd = np.hstack([ref["U"], ref["Z"]])
    assert np.linalg.norm(X - Xd) <= 1e-8 * np.linalg.norm(Xd)
    _, its, _ = osol.pcg_jacobi_multi(ref["A"], rhs, 1e-12)
    if precond == "jacobi" or levels == 0:
        # iteration counts follow the oracle's Jacobi-PCG
        assert np.all(np.abs(res.iters - its) <= np.maximum(2, 0.03 * its)), (res.iters, its)
    else:
        # the V-cycle takes at most a fifth of Jacobi-PCG's iterations
        assert np.all(5 * res.iters <= its), (res.iters, its)


@pytest.mark.parametrize("precond", ["auto", "jacobi"])
@pytest.mark.parametrize("name", ["t3d_b", "t3d_c", "t2d"])
def test_solve_mixed_reaches_fp64_accuracy(dotlib, dev, name, precond):
    wl, prob, W, V, data, ref = case(name)
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    pc = dotlib.DOT_PRECOND_AUTO if precond == "auto" else dotlib.DOT_PRECOND_JACOBI
    with op:
        op.pals_mua(pals, th)
        rhs = np.hstack([ref["BW"], ref["CV"]])
        res = op.solve(torch.tensor(rhs, device=dev), rtol=1e-10, precision=dotlib.DOT_MIXED,
                       inner_rtol=0.1, precond=pc)
        X = res.x.cpu().numpy()
    assert res.converged and res.outer >= 1
    true_rel = osol.relative_residuals(ref["A"], X, rhs)
    assert np.all(true_rel <= 1e-10), true_rel.max()
    Xd = np.hstack([ref["U"], ref["Z"]])
    assert np.linalg.norm(X - Xd) <= 1e-6 * np.linalg.norm(Xd)


@pytest.mark.parametrize("name", ["t3d_c", "t3d_b"])
def test_solve_bitwise_deterministic(dotlib, dev, name):
    wl, prob, W, V, data, ref = case(name)
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    with op:
        op.pals_mua(pals, th)
        rhs = torch.tensor(np.hstack([ref["BW"], ref["CV"]]), device=dev)
        for prec in (dotlib.DOT_FP64, dotlib.DOT_MIXED):
            a = op.solve(rhs, rtol=1e-10, precision=prec)
            b = op.solve(rhs, rtol=1e-10, precision=prec)
            assert torch.equal(a.x, b.x)
            assert np.array_equal(a.iters, b.iters)


def test_solve_edge_cases(dotlib, dev):
    wl, prob, W, V, data, ref = case("t3d")
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    with op:
        op.pals_mua(pals, th)
        # single column, and a zero column among others
        rhs = np.zeros((prob.N, 3))
        rhs[:, 0] = ref["BW"][:, 0]
        rhs[:, 2] = ref["CV"][:, 1]
        res = op.solve(torch.tensor(rhs, device=dev), rtol=1e-12)
        X = res.x.cpu().numpy()
        assert res.converged and np.all(X[:, 1] == 0.0) and res.iters[1] == 0
        assert res.relres[1] == 0.0
        one = op.solve(torch.tensor(rhs[:, :1].copy(), device=dev), rtol=1e-12)
        assert np.array_equal(one.x.cpu().numpy()[:, 0], X[:, 0])
        # iteration cap: outputs valid, status "not converged"
        with pytest.warns(dotlib.NotConverged):
            capped = op.solve(torch.tensor(rhs, device=dev), rtol=1e-12, max_iter=3)
        assert not capped.converged and capped.iters_max == 3
        # non-finite data is reported
        bad = rhs.copy()
        bad[5, 0] = np.nan
        with pytest.raises(dotlib.DotError) as ei:
            op.solve(torch.tensor(bad, device=dev), rtol=1e-12)
        assert ei.value.code == -5


@pytest.mark.parametrize("shape", ["t3d_b", (32, 16, 8), (64, 64, 64), "t3d", "t3d_c", "t2d", "C1"])
def test_multigrid_vcycle_matches_reference_model(dotlib, dev, shape):
    """One binary64 V-cycle (as an approximate inverse of A) against the
    scipy model of the V-cycle on random right-hand sides, 5 columns (a ragged column
    group); grids cubic with mixed boundary faces, flat (one tile across x,
    two coarse levels), 64^3, odd sides in every direction (ragged last
    aggregates, an odd number of planes per level) and 2D."""
    import mg_reference as omg
    if isinstance(shape, str):
        wl = synthetic.make_workload(synthetic.get_config(shape))
    else:
        wl = synthetic.make_workload(synthetic.get_config("C2", n=shape))
    prob = oprob.build(wl)
    mua = prob.mua(wl.theta_ref)
    lv = omg.hierarchy(prob.n, prob.bc, prob.D, mua)
    rng = np.random.default_rng(11)
    R = rng.standard_normal((prob.N, 5))
    Zr = omg.apply(lv, R)
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    with op:
        op.pals_mua(pals, th)
        assert op.multigrid_levels == len(lv)
        Z = op.multigrid_apply(torch.tensor(R, device=dev)).cpu().numpy()
    err = np.linalg.norm(Z - Zr, axis=0) / np.linalg.norm(Zr, axis=0)
    print(f"[mg {shape}] levels {len(lv)} max rel err {err.max():.2e}", flush=True)
    assert np.all(err <= 1e-12), err


def test_multigrid_availability(dotlib, dev):
    """No hierarchy where a side has fewer than 5 cells (a coarse side would
    fall below 3): the solver falls back to Jacobi and an explicit request
    is refused."""
    for name, n in (("t3d", (19, 13, 4)), ("t2d", (37, 4))):
        wl = synthetic.make_workload(synthetic.get_config(name, n=n))
        op, grid, pals, th = gpu_operator(dotlib, dev, wl)
        with op:
            op.pals_mua(pals, th)
            assert op.multigrid_levels == 0
            b = torch.zeros((int(np.prod(n)), 1), dtype=torch.float64, device=dev)
            b[0, 0] = 1.0
            with pytest.raises(dotlib.DotError) as ei:
                op.solve(b, rtol=1e-8, precond=dotlib.DOT_PRECOND_MG)
            assert ei.value.code == -1
            with pytest.raises(dotlib.DotError):
                op.multigrid_apply(b)


@pytest.mark.parametrize("name", ["t3d", "t3d_b"])
def test_indefinite_operator_reports_breakdown(dotlib, dev, name):
    """An indefinite A is reported as a CG breakdown; on a grid with a
    hierarchy the coarse diagonals turn negative first, so the solver
    drops the V-cycle (no longer positive definite) and uses Jacobi."""
    wl, prob, W, V, data, ref = case(name)
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    with op:
        # a strongly negative absorption in the interior makes A indefinite
        # while keeping its diagonal positive
        mu = np.full(prob.N, 0.01)
        h = prob.h
        x = prob.x
        centre = np.all(np.abs(x - x.mean(axis=0)) < 0.2, axis=1)
        diag_pos = 2.0 * 3 * h * prob.D.min() / h ** 3 * 0.9
        mu[centre] = -diag_pos
        op.set_mua(torch.tensor(mu, device=dev))
        assert op.multigrid_levels == 0
        A = odisc.assemble(prob.n, prob.bc, prob.D, mu)
        assert A.diagonal().min() > 0
        rng = np.random.default_rng(3)
        b = rng.standard_normal((prob.N, 2))
        with pytest.raises(dotlib.DotError) as ei:
            op.solve(torch.tensor(b, device=dev), rtol=1e-12, max_iter=5000)
        assert ei.value.code == -4


@pytest.mark.parametrize("name", NAMES)
def test_sampled_misfit_matches_oracle(dotlib, dev, name):
    wl, prob, W, V, data, ref = case(name)
    op, *_ = gpu_operator(dotlib, dev, wl)
    with op:
        U = torch.tensor(ref["U"], device=dev)
        Rs, f = op.sampled_misfit(wl.det_cells, U, torch.tensor(V, device=dev),
                                  torch.tensor(data @ W, device=dev))
    assert np.linalg.norm(Rs.cpu().numpy() - ref["Rs"]) <= 1e-12 * np.linalg.norm(ref["Rs"])
    assert f == pytest.approx(ref["f"], rel=1e-12)


@pytest.mark.parametrize("name", NAMES)
def test_jacobian_fp64_matches_oracle(dotlib, dev, name):
    wl, prob, W, V, data, ref = case(name)
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    with op:
        op.pals_mua(pals, th)
        Js = op.jacobian(torch.tensor(ref["U"], device=dev), torch.tensor(ref["Z"], device=dev),
                         dotlib.DOT_JAC_FP64).cpu().numpy()
    Jr = ref["Js"]
    assert Js.shape == Jr.shape
    assert np.linalg.norm(Jr) > 0
    assert np.linalg.norm(Js - Jr) <= 1e-12 * np.linalg.norm(Jr)


@pytest.mark.parametrize("ls,ld", [(64, 64), (3, 70), (9, 64)])
def test_jacobian_large_sample_counts(dotlib, dev, ls, ld):
    """Sample counts at and beyond one pass of the matrix-core kernels, against
    the oracle's loop nest on random fields (the contraction is linear in
    them): 64 x 64 (binary64 in detector tiles of 51, the split forms at their
    largest tiling), l_d = 70 (ragged l_s + l_d = 73; the split forms in two
    detector tiles) and 9 x 64 (one row tile, four detector tiles)."""
    wl = synthetic.make_workload(synthetic.get_config("t3d"))
    prob = oprob.build(wl)
    rng = np.random.default_rng(ls * 100 + ld)
    U = rng.standard_normal((prob.N, ls))
    Z = rng.standard_normal((prob.N, ld))
    Jr = oest.jacobian_sparse_loops(U, Z, prob.G(wl.theta_ref))
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    with op:
        op.pals_mua(pals, th)
        Ut, Zt = torch.tensor(U, device=dev), torch.tensor(Z, device=dev)
        Js = op.jacobian(Ut, Zt, dotlib.DOT_JAC_FP64).cpu().numpy()
        assert np.linalg.norm(Js - Jr) <= 1e-12 * np.linalg.norm(Jr)
        # three parts (the product form): binary32-level operands, within
        # the 1e-6 bound; two parts (the faster option): each product is
        # exact to about 2^-16 relative (dropped lo lo term and lo
        # rounding), within its stated 2e-5 bound
        J2 = op.jacobian(Ut, Zt, dotlib.DOT_JAC_SPLIT_BF16).cpu().numpy()
        J3 = op.jacobian(Ut, Zt, dotlib.DOT_JAC_SPLIT_BF16X3).cpu().numpy()
        e2 = np.linalg.norm(J2 - Jr) / np.linalg.norm(Jr)
        e3 = np.linalg.norm(J3 - Jr) / np.linalg.norm(Jr)
        print(f"[jac {ls}x{ld}] 3-part {e3:.2e}, 2-part option {e2:.2e}", flush=True)
        assert e3 <= 1e-6
        assert e2 <= 2e-5


@pytest.mark.parametrize("name", NAMES)
def test_gradient_matches_oracle(dotlib, dev, name):
    wl, prob, W, V, data, ref = case(name)
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    with op:
        op.pals_mua(pals, th)
        g = op.grad_misfit(torch.tensor(ref["U"], device=dev), torch.tensor(ref["Z"], device=dev),
                           torch.tensor(ref["Rs"], device=dev)).cpu().numpy()
    assert np.linalg.norm(g - ref["g"]) <= 1e-12 * np.linalg.norm(ref["g"])


def test_reciprocity_on_gpu(dotlib, dev):
    """Co-located optodes and A = A^T: the GPU measurement matrix is symmetric."""
    wl, prob, W, V, data, ref = case("C1")
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    with op:
        op.pals_mua(pals, th)
        B = op.form_rhs(wl.src_cells, torch.eye(16, dtype=torch.float64, device=dev))
        X = op.solve(B, rtol=1e-13).x.cpu().numpy()
    M = X[wl.det_cells, :]
    assert np.linalg.norm(M - M.T) <= 1e-11 * np.linalg.norm(M)


def test_gemm_matches_numpy(dotlib, dev):
    rng = np.random.default_rng(9)
    for (m, k, n) in [(7, 5, 3), (40, 300, 33), (17, 1, 19)]:
        A, B = rng.standard_normal((m, k)), rng.standard_normal((k, n))
        for ta in (False, True):
            for tb in (False, True):
                Aa = A.T.copy() if ta else A
                Bb = B.T.copy() if tb else B
                C = dotlib.gemm(torch.tensor(Aa, device=dev), torch.tensor(Bb, device=dev), ta, tb)
                assert np.allclose(C.cpu().numpy(), A @ B, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("name", NAMES)
def test_jacobian_split_bf16_error(dotlib, dev, name):
    """Split-bfloat16 contraction against the oracle's binary64 loop nest on
    identical fields: the 3-part form (the product form) within the 1e-6
    relative Frobenius bound on every parity grid; the 2-part option within
    its stated 2e-5 (2^-16 per product, averaged over the band cells)."""
    wl, prob, W, V, data, ref = case(name)
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    with op:
        op.pals_mua(pals, th)
        U = torch.tensor(ref["U"], device=dev)
        Z = torch.tensor(ref["Z"], device=dev)
        J2 = op.jacobian(U, Z, dotlib.DOT_JAC_SPLIT_BF16).cpu().numpy()
        J3 = op.jacobian(U, Z, dotlib.DOT_JAC_SPLIT_BF16X3).cpu().numpy()
    Jr = ref["Js"]
    e2 = np.linalg.norm(J2 - Jr) / np.linalg.norm(Jr)
    e3 = np.linalg.norm(J3 - Jr) / np.linalg.norm(Jr)
    print(f"{name}: 3-part rel err {e3:.3e}, 2-part option {e2:.3e}")
    assert e3 <= 1e-6
    assert e2 <= 2e-5


@pytest.mark.parametrize("check_every", [1, 2])
def test_mixed_multigrid_iteration_cap(dotlib, dev, check_every):
    """Binary32 CG with the multigrid preconditioner stopped by the iteration
    cap: the flags are read one poll late and the last correction is folded
    into x at the end, so the returned x carries every iteration (its
    residual, recomputed by the oracle's operator, is far below the first
    one's and equals the reported one) and the status is "not converged"."""
    wl, prob, W, V, data, ref = case("t3d_b")
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    with op:
        op.pals_mua(pals, th)
        assert op.multigrid_levels == 4   # 24^3 down to 3^3
        rhs = np.hstack([ref["BW"], ref["CV"]])
        # binary32 V-cycle vectors, so that the iterates follow the binary64
        # model closely (bfloat16 storage steers CG slightly differently)
        with pytest.warns(dotlib.NotConverged):
            capped = op.solve(torch.tensor(rhs, device=dev), rtol=1e-14, max_iter=3,
                              precision=dotlib.DOT_MIXED, check_every=check_every,
                              precond=dotlib.DOT_PRECOND_MG_F32)
        X = capped.x.cpu().numpy()
    assert not capped.converged and capped.iters_max == 3
    true_rel = osol.relative_residuals(ref["A"], X, rhs)
    assert np.allclose(true_rel, capped.relres, rtol=1e-6, atol=1e-15)
    # CG preconditioned with the scipy V-cycle model, after the same 3 iterations
    import mg_reference as omg
    A = ref["A"]
    lv = omg.hierarchy(prob.n, prob.bc, prob.D, prob.mua(wl.theta_ref))
    want = []
    for j in range(rhs.shape[1]):
        b = rhs[:, j]
        x = np.zeros_like(b)
        r = b.copy()
        z = omg.apply(lv, r)
        p = z.copy()
        rho = r @ z
        for _ in range(3):
            w = A @ p
            al = rho / (p @ w)
            x += al * p
            r -= al * w
            z = omg.apply(lv, r)
            rn = r @ z
            p = z + (rn / rho) * p
            rho = rn
        want.append(np.linalg.norm(b - A @ x) / np.linalg.norm(b))
    assert np.allclose(true_rel, want, rtol=1e-3), (true_rel.max(), max(want))


def test_multigrid_refreshed_by_new_parameters(dotlib, dev):
    """A second dot_pals_mua on the same operator rebuilds every level of the
    hierarchy (coefficients, sqrt(diag) in both precisions, prolongation
    weights): an iteration-capped mixed multigrid solve after it equals the
    same solve on a fresh operator built for the new parameters, and differs
    from the solve before the update."""
    wl, prob, W, V, data, ref = case("t3d_b")
    rhs = torch.tensor(np.hstack([ref["BW"], ref["CV"]]), device=dev)

    def capped(op):
        with pytest.warns(dotlib.NotConverged):
            return op.solve(rhs, rtol=1e-14, max_iter=3, precision=dotlib.DOT_MIXED,
                            precond=dotlib.DOT_PRECOND_MG).x.cpu().numpy()

    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    # moved RBF centres: a different absorption on every level
    th2 = th.clone().reshape(-1, 2 + grid.dim)
    th2[:, 2:] += 0.05
    th2 = th2.reshape(-1)
    with op:
        op.pals_mua(pals, th)
        X1 = capped(op)
        op.pals_mua(pals, th2)
        X2 = capped(op)
    fresh, *_ = gpu_operator(dotlib, dev, wl)
    with fresh:
        fresh.pals_mua(pals, th2)
        Xf = capped(fresh)
    scale = np.linalg.norm(Xf)
    print(f"[mg refresh] |X2 - Xf| {np.linalg.norm(X2 - Xf) / scale:.2e} "
          f"|X1 - Xf| {np.linalg.norm(X1 - Xf) / scale:.2e}", flush=True)
    assert np.linalg.norm(X2 - Xf) <= 1e-12 * scale
    assert np.linalg.norm(X1 - Xf) > 1e-4 * scale


@pytest.mark.parametrize("name", ["t3d_b", "t3d_c", "t2d", (64, 64, 64)])
def test_mixed_vcycle_storage_bf16_vs_binary32(dotlib, dev, name):
    """The mixed solve with the V-cycle's work vectors in bfloat16 (the
    default) and in binary32: both reach relres 1e-10 (recomputed with the
    oracle's CSR operator) and the narrower storage costs at most one
    iteration, in the maximum and in the mean over columns (iterations
    counted exactly: the flags are polled every iteration)."""
    if isinstance(name, str):
        wl, prob, W, V, data, ref = case(name)
        A, rhs = ref["A"], np.hstack([ref["BW"], ref["CV"]])
    else:
        wl = synthetic.make_workload(synthetic.get_config("C2", n=name))
        prob = oprob.build(wl)
        A = prob.operator(wl.theta_ref)
        Wm, Vm = oest.sample_matrix(wl.w_signs), oest.sample_matrix(wl.v_signs)
        rhs = np.hstack([oest.simultaneous_rhs(prob.N, wl.src_cells, Wm),
                         oest.simultaneous_rhs(prob.N, wl.det_cells, Vm)])
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    out = {}
    with op:
        op.pals_mua(pals, th)
        assert op.multigrid_levels >= 2
        for pc in (dotlib.DOT_PRECOND_MG, dotlib.DOT_PRECOND_MG_F32):
            res = op.solve(torch.tensor(rhs, device=dev), rtol=1e-10, precision=dotlib.DOT_MIXED,
                           inner_rtol=0.01, precond=pc, check_every=1)
            assert res.converged
            X = res.x.cpu().numpy()
            true_rel = osol.relative_residuals(A, X, rhs)
            assert np.all(true_rel <= 1e-10), true_rel.max()
            out[pc] = res.iters
    print(f"[mg storage {name}] iterations bf16 {out[dotlib.DOT_PRECOND_MG]} "
          f"binary32 {out[dotlib.DOT_PRECOND_MG_F32]}", flush=True)
    it_h, it_s = out[dotlib.DOT_PRECOND_MG], out[dotlib.DOT_PRECOND_MG_F32]
    assert it_h.max() <= it_s.max() + 1 and it_h.mean() <= it_s.mean() + 1


def test_profile_kinds_select_timed_launches(dotlib, dev):
    """dot_profile_kinds: only the selected kinds are timed, profile_enable
    selects every kind again, and the solve itself is unchanged."""
    wl, prob, W, V, data, ref = case("t3d_b")
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    rhs = torch.tensor(np.hstack([ref["BW"], ref["CV"]]), device=dev)
    with op:
        with pytest.raises(dotlib.DotError):
            op.profile_kinds(dotlib.DOT_PROF_PCG2_FP32)
        op.pals_mua(pals, th)
        assert op.multigrid_levels >= 2

        def solve():
            return op.solve(rhs, rtol=1e-10, precision=dotlib.DOT_MIXED, inner_rtol=0.01)

        op.profile_enable(True)
        op.profile_kinds(dotlib.DOT_PROF_PCG2_FP32)
        r1 = solve()
        ms2, n2, c2 = op.profile_read(dotlib.DOT_PROF_PCG2_FP32)
        assert n2 >= r1.iters_max and ms2 > 0.0 and c2 >= n2
        for kind in (dotlib.DOT_PROF_PCG1_FP32, dotlib.DOT_PROF_VCYCLE_FP32, dotlib.DOT_PROF_RESID):
            assert op.profile_read(kind) == (0.0, 0, 0)
        op.profile_enable(True)
        r2 = solve()
        for kind in (dotlib.DOT_PROF_PCG1_FP32, dotlib.DOT_PROF_PCG2_FP32,
                     dotlib.DOT_PROF_VCYCLE_FP32, dotlib.DOT_PROF_RESID):
            assert op.profile_read(kind)[1] > 0
        op.profile_enable(False)
    assert torch.equal(r1.x, r2.x)


def test_mixed_solve_scales_with_the_right_hand_side(dotlib, dev):
    """The binary32 residual is kept at scale |b^| per column: right-hand
    sides scaled by 1e-20 and 1e20 (and a block mixing both) converge and
    give the scaled solutions."""
    wl, prob, W, V, data, ref = case("t3d_b")
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    rhs = np.hstack([ref["BW"], ref["CV"]])
    with op:
        op.pals_mua(pals, th)

        def solve(b):
            res = op.solve(torch.tensor(b, device=dev), rtol=1e-10, precision=dotlib.DOT_MIXED,
                           inner_rtol=0.01)
            assert res.converged
            X = res.x.cpu().numpy()
            assert np.all(osol.relative_residuals(ref["A"], X, b) <= 1e-10)
            return X

        X1 = solve(rhs)
        for f in (1e-20, 1e20):
            Xf = solve(rhs * f)
            assert np.linalg.norm(Xf / f - X1) <= 1e-7 * np.linalg.norm(X1)
        mixed = rhs.copy()
        mixed[:, 0] *= 1e-20
        mixed[:, 1] *= 1e20
        Xm = solve(mixed)
        assert np.linalg.norm(Xm[:, 2:] - X1[:, 2:]) <= 1e-7 * np.linalg.norm(X1[:, 2:])


@pytest.mark.parametrize("precond", ["mg", "jacobi"])
def test_mixed_solve_ignores_stale_workspace_and_output(dotlib, dev, precond):
    """The binary32 CG does not clear x^, its correction or the first
    direction at set-up (per-column flags mark them as unset): a workspace
    and an output block full of NaN bit patterns give bit-identical
    solutions, iteration counts and residuals to zero-filled ones, for
    converged columns, a zero right-hand side and columns stopped by the
    iteration cap."""
    wl, prob, W, V, data, ref = case("t3d_b")
    op, grid, pals, th = gpu_operator(dotlib, dev, wl)
    rhs = np.hstack([ref["BW"], ref["CV"]])
    rhs[:, 1] = 0.0
    pc = dotlib.DOT_PRECOND_MG if precond == "mg" else dotlib.DOT_PRECOND_JACOBI
    B = torch.tensor(rhs, device=dev).t().contiguous().t()
    with op:
        op.pals_mua(pals, th)
        nbytes = op.solve_workspace_bytes(B.shape[1], dotlib.DOT_MIXED)

        def run(fill, **kw):
            work = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
            work = work[(-work.data_ptr()) % 256:]
            work.fill_(fill)
            out = torch.empty_like(B).t().contiguous().t()
            out.t().view(torch.uint8).fill_(fill)
            res = op.solve(B, precision=dotlib.DOT_MIXED, precond=pc, out=out, work=work,
                           inner_rtol=0.01, warn=False, **kw)
            torch.cuda.synchronize()
            return res

        for kw in ({"rtol": 1e-10}, {"rtol": 1e-14, "max_iter": 3}):
            clean, stale = run(0, **kw), run(255, **kw)
            assert torch.isfinite(stale.x).all()
            assert torch.equal(clean.x, stale.x), kw
            assert np.array_equal(clean.iters, stale.iters)
            assert np.array_equal(clean.relres, stale.relres)
            assert torch.count_nonzero(stale.x[:, 1]) == 0
        assert clean.iters_max == 3 and not clean.converged
