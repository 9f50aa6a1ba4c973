"""GPU parity at the remaining workload sizes and for the estimator's theorems:

  * 64^3 (64/64 optodes, l = 8, 27 RBFs): binary64 CG with Jacobi
    preconditioning and with the V-cycle to relres 1e-10, every column's
    residual recomputed by the oracle's CSR operator; all 108 columns of the
    8 x 8 x 108 sampled Jacobian against the oracle's sparse loop nest on the
    GPU fields, and the 135-parameter variant (width active as well);
  * 96^3 workload layout (16 x 8 optodes, l = 16, 100 RBFs, 500 params):
    the autograd gradient against the oracle's gradient computed from its own
    direct solve on a 24^3 grid with the same phantom layout, and at 96^3
    against the oracle's adjoint form on sampled RBF columns of the GPU
    fields, plus central differences with a per-entry tolerance;
  * Thm 3.1 on the GPU sampled misfit: over the complete set of Rademacher
    sample vectors it equals ||R||_F^2 exactly (to rounding), and the Monte
    Carlo mean over seeded single-sample draws lies within a CLT bound whose
    variance is enumerated exactly on the CPU;
  * a negative RBF width parameter beta (the support depends on beta^2):
    Jacobian and gradient against the oracle;
  * bitwise rerun determinism of J_s (all three forms) and of the gradient.
"""

import numpy as np
import pytest
import torch

import synthetic
from oracle import estimators as oest
from oracle import problem as oprob
from oracle import solvers as osol
from oracle_columns import support_columns

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dl():
    import paper_1706_05586_amd as m
    return m


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


def gpu_fields(dl, dev, wl, theta, precision, rtol, precond=0):
    cfg = wl.cfg
    grid, pals = dl.Grid.from_config(cfg), dl.Pals.from_config(cfg)
    _, D = dl.pals_field(grid, pals, torch.tensor(wl.theta_ref, device=dev), cfg.mus_prime)
    op = dl.Operator(grid, D)
    op.pals_mua(pals, torch.tensor(theta, device=dev))
    W = torch.tensor(oest.sample_matrix(wl.w_signs), device=dev)
    V = torch.tensor(oest.sample_matrix(wl.v_signs), device=dev)
    ls, ld = W.shape[1], V.shape[1]
    rhs = dl.empty_colmajor(grid.N, ls + ld, dev)
    op.form_rhs(wl.src_cells, W, out=rhs[:, :ls])
    op.form_rhs(wl.det_cells, V, out=rhs[:, ls:])
    res = op.solve(rhs, rtol=rtol, precision=precision, precond=precond)
    return op, W, V, rhs, res


@pytest.mark.parametrize("active", [5, 7])
def test_64cubed_jacobi_pcg_and_full_sampled_jacobian(dl, dev, active):
    """The 64^3 workload: 27 RBFs with (alpha, chi) active = 108 parameters,
    and the variant with the width as well (27 x 5 = 135)."""
    cfg = synthetic.get_config("C2", active=active)
    wl = synthetic.make_workload(cfg)
    prob = oprob.build(wl)
    A = prob.operator(wl.theta_ref)
    ls = cfg.l_s
    for precond in (dl.DOT_PRECOND_JACOBI, dl.DOT_PRECOND_AUTO):
        say(f"[C2 active={active}] binary64 solve, precond {precond}")
        op, W, V, rhs, res = gpu_fields(dl, dev, wl, wl.theta_ref, dl.DOT_FP64, 1e-10, precond)
        X, B = res.x.cpu().numpy(), rhs.cpu().numpy()
        rel = osol.relative_residuals(A, X, B)
        say(f"[C2] iters {res.iters_max} true relres max {rel.max():.2e}")
        assert res.converged and np.all(rel <= 1.5e-10), rel.max()
        assert np.allclose(rel, res.relres, rtol=1e-3, atol=1e-14)
        if precond == dl.DOT_PRECOND_AUTO:
            assert op.multigrid_levels >= 3
        else:
            prec_iters = res.iters_max
    assert res.iters_max * 10 < prec_iters   # the V-cycle against Jacobi
    with op:
        U, Z = res.x[:, :ls], res.x[:, ls:]
        J64 = op.jacobian(U, Z, dl.DOT_JAC_FP64).cpu().numpy()
        J3 = op.jacobian(U, Z, dl.DOT_JAC_SPLIT_BF16X3).cpu().numpy()
    G = prob.G(wl.theta_ref)
    assert G.shape[1] == cfg.n_p == J64.shape[1] == (108 if active == 5 else 135)
    Jr = oest.jacobian_sparse_loops(X[:, :ls], X[:, ls:], G)
    e64 = np.linalg.norm(J64 - Jr) / np.linalg.norm(Jr)
    e3 = np.linalg.norm(J3 - Jr) / np.linalg.norm(Jr)
    col = np.linalg.norm(J64 - Jr, axis=0) / np.maximum(np.linalg.norm(Jr, axis=0), 1e-300)
    say(f"[C2 active={active}] J64 {e64:.2e} (worst column {col.max():.2e}), 3-part split {e3:.2e}")
    assert e64 <= 1e-12 and col.max() <= 1e-10
    assert e3 <= 1e-6


def misfit_problem(dl, dev, wl, data, rtol=1e-12):
    cfg = wl.cfg
    grid, pals = dl.Grid.from_config(cfg), dl.Pals.from_config(cfg)
    th = torch.tensor(wl.theta_ref, device=dev)
    _, D = dl.pals_field(grid, pals, th, cfg.mus_prime)
    op = dl.Operator(grid, D)
    W = torch.tensor(oest.sample_matrix(wl.w_signs), device=dev)
    V = torch.tensor(oest.sample_matrix(wl.v_signs), device=dev)
    DW = dl.gemm(torch.tensor(data, device=dev), W)
    return dl.MisfitProblem(op=op, pals=pals, theta=th, src_cells=wl.src_cells,
                            det_cells=wl.det_cells, W=W, V=V, DW=DW, rtol=rtol)


def autograd_gradient(dl, prob):
    p = prob.params_of(prob.theta).clone().requires_grad_(True)
    f = dl.misfit(p, prob)
    f.backward()
    return f.item(), p.grad.detach().cpu().numpy()


def test_96cubed_layout_gradient_against_oracle_direct_solve(dl, dev):
    """The differentiation workload's phantom layout (100 RBFs on a 5 x 5 x 4
    lattice, 500 parameters, 16 x 8 optodes, l = 16) on a 24^3 grid, where the
    oracle solves directly: autograd gradient against the oracle gradient."""
    cfg = synthetic.get_config("C4", n=(24, 24, 24))
    wl = synthetic.make_workload(cfg)
    oprb = oprob.build(wl)
    data = oprob.synthetic_data(oprb, wl)
    W, V = oest.sample_matrix(wl.w_signs), oest.sample_matrix(wl.v_signs)
    ref = oprob.evaluate(oprb, wl, wl.theta_ref, W, V, data)
    prob = misfit_problem(dl, dev, wl, data)
    with prob.op:
        f, g = autograd_gradient(dl, prob)
    err = np.linalg.norm(g - ref["g"]) / np.linalg.norm(ref["g"])
    say(f"[C4 layout 24^3] n_p {g.size} f {f:.6e} vs {ref['f']:.6e}, gradient rel err {err:.2e}")
    assert g.size == 500
    assert f == pytest.approx(ref["f"], rel=1e-10)
    assert err <= 1e-7


def test_96cubed_gradient_sampled_columns_and_central_differences(dl, dev):
    """96^3: the autograd gradient against the oracle's adjoint form on the
    GPU fields (whose residuals the oracle checks) for sampled RBFs, and
    against central differences (step 1e-6) entry by entry."""
    cfg = synthetic.get_config("C4")
    wl = synthetic.make_workload(cfg)
    # data from every source at theta_true, solved by the library itself
    grid, pals = dl.Grid.from_config(cfg), dl.Pals.from_config(cfg)
    _, D = dl.pals_field(grid, pals, torch.tensor(wl.theta_ref, device=dev), cfg.mus_prime)
    with dl.Operator(grid, D) as op0:
        op0.pals_mua(pals, torch.tensor(wl.theta_true, device=dev))
        B = op0.form_rhs(wl.src_cells, torch.eye(cfg.n_s, dtype=torch.float64, device=dev))
        M = op0.solve(B, rtol=1e-12).x.cpu().numpy()[wl.det_cells, :]
        del B
    data = M * (1.0 + cfg.noise * wl.xi)
    prob = misfit_problem(dl, dev, wl, data)
    ls = cfg.l_s
    with prob.op:
        f0, g = autograd_gradient(dl, prob)
        # the same fields (the solves are bitwise deterministic) and R_s
        U, Z = prob.forward_fields(True)
        Rs, f1 = prob.op.sampled_misfit(wl.det_cells, U, prob.V, prob.DW)
        assert f1 == f0
        X = torch.cat([U, Z], dim=1).cpu().numpy()
        rhs = prob.op.form_rhs(wl.src_cells, prob.W).cpu().numpy()
        rhs = np.hstack([rhs, prob.op.form_rhs(wl.det_cells, prob.V).cpu().numpy()])
        A = oprob.build(wl).operator(wl.theta_ref)
        rel = osol.relative_residuals(A, X, rhs)
        say(f"[C4 96^3] true relres max {rel.max():.2e}")
        assert np.all(rel <= 1.5e-12)
        Rn = Rs.cpu().numpy()
        Rs_def = oest.sampled_residual(X[:, :ls], wl.det_cells, prob.V.cpu().numpy(),
                                       data @ prob.W.cpu().numpy())
        assert np.linalg.norm(Rn - Rs_def) <= 1e-12 * np.linalg.norm(Rs_def)
        for m in (0, 33, 67, 99):
            cells, G, na = support_columns(wl, m)
            gr = oest.gradient_adjoint(X[cells, :ls], X[cells, ls:], Rn, G)
            sl = slice(m * na, (m + 1) * na)
            e = np.linalg.norm(g[sl] - gr) / np.linalg.norm(gr)
            say(f"[C4 96^3] RBF {m}: gradient rel err {e:.2e}")
            assert e <= 1e-11
        params = prob.params_of(prob.theta)
        order = np.argsort(-np.abs(g))
        sample = [int(k) for k in list(order[:4]) + list(order[100:103]) + list(order[250:252])]
        h = 1e-6
        # each evaluation of f carries a relative error of about the solver's
        # tolerance (1e-12), so the central difference has an absolute noise
        # floor of about 1e-12 |f| / h besides its relative truncation error
        noise = 1e-12 * abs(f0) / h
        say(f"[C4 96^3] f {f0:.6e}, central-difference noise floor {noise:.2e}")
        for k in sample:
            e = torch.zeros_like(params)
            e[k] = h
            fp = dl.misfit(params + e, prob).item()
            fm = dl.misfit(params - e, prob).item()
            fd = (fp - fm) / (2 * h)
            say(f"[C4 96^3] FD param {k}: g {g[k]:.9e} fd {fd:.9e} rel {abs(fd - g[k]) / abs(g[k]):.2e}")
            assert abs(fd - g[k]) <= 2e-5 * abs(g[k]) + noise, (k, fd, g[k])


def _signs(n):
    """All 2^n Rademacher vectors of length n as columns (n x 2^n)."""
    idx = np.arange(2 ** n)
    return np.where((idx[None, :] >> np.arange(n)[:, None]) & 1, -1.0, 1.0)


def test_theorem_3_1_on_gpu_sampled_misfit(dl, dev):
    """E ||V^T R W||_F^2 = ||R||_F^2 (Thm 3.1).  With W and V holding every
    Rademacher vector (2^8 each, scaled by 2^-4) the GPU sampled misfit is the
    exact expectation; single-sample draws average to ||R||_F^2 within five
    standard errors of the exactly enumerated variance."""
    wl = synthetic.make_workload(synthetic.get_config("t3d"))
    prob = oprob.build(wl)
    data = oprob.synthetic_data(prob, wl)
    A = prob.operator(wl.theta_ref)
    M = oest.measurements(A, prob.n, wl.src_cells, wl.det_cells)
    R = M - data
    cfg = wl.cfg
    grid, pals = dl.Grid.from_config(cfg), dl.Pals.from_config(cfg)
    _, D = dl.pals_field(grid, pals, torch.tensor(wl.theta_ref, device=dev), cfg.mus_prime)
    with dl.Operator(grid, D) as op:
        op.pals_mua(pals, torch.tensor(wl.theta_ref, device=dev))
        n_s = len(wl.src_cells)
        B = op.form_rhs(wl.src_cells, torch.eye(n_s, dtype=torch.float64, device=dev))
        UI = op.solve(B, rtol=1e-13).x                       # A^-1 B, every source
        Dt = torch.tensor(data, device=dev)
        # exact expectation over 8 sources and 8 detectors
        s8, d8 = np.arange(8), np.arange(8)
        S = _signs(8) / 16.0
        St = torch.tensor(S, device=dev)
        U8 = dl.gemm(UI[:, s8].contiguous(), St)
        DW8 = dl.gemm(Dt[d8][:, s8].contiguous(), St)
        _, f = op.sampled_misfit(wl.det_cells[d8], U8, St, DW8)
        R8 = R[np.ix_(d8, s8)]
        exact = float(np.sum(R8 ** 2))
        say(f"[Thm 3.1] full enumeration: 2f = {2 * f:.15e}, ||R||^2 = {exact:.15e}")
        assert 2 * f == pytest.approx(exact, rel=1e-9)
        # Monte Carlo over single-sample draws, all 12 sources and detectors
        n_d = len(wl.det_cells)
        rng = np.random.default_rng(31)
        draws = 4000
        vals = np.empty(draws)
        for t in range(draws):
            w = rng.choice([-1.0, 1.0], size=(n_s, 1))
            v = rng.choice([-1.0, 1.0], size=(n_d, 1))
            wt, vt = torch.tensor(w, device=dev), torch.tensor(v, device=dev)
            _, ft = op.sampled_misfit(wl.det_cells, dl.gemm(UI, wt), vt, dl.gemm(Dt, wt))
            vals[t] = 2.0 * ft
    # exact mean and variance of (v^T R w)^2 over all 2^12 x 2^12 pairs
    Sw, Sv = _signs(n_s), _signs(n_d)
    q = (Sv.T @ R @ Sw) ** 2
    mean, var = q.mean(), q.var()
    assert mean == pytest.approx(np.sum(R ** 2), rel=1e-12)
    se = np.sqrt(var / draws)
    say(f"[Thm 3.1] MC mean {vals.mean():.6e}, ||R||^2 {mean:.6e}, standard error {se:.2e}")
    assert abs(vals.mean() - mean) <= 5.0 * se


def test_negative_width_parameter(dl, dev):
    """beta enters the PaLS level set squared: flipping its sign for some
    RBFs leaves mu unchanged and flips the sign of d mu / d beta only; the
    Jacobian and gradient follow the oracle."""
    wl = synthetic.make_workload(synthetic.get_config("t3d"))
    th = wl.theta_ref.copy()
    th[::2, 1] *= -1.0
    prob = oprob.build(wl)
    data = oprob.synthetic_data(prob, wl)
    W, V = oest.sample_matrix(wl.w_signs), oest.sample_matrix(wl.v_signs)
    ref = oprob.evaluate(prob, wl, th, W, V, data)
    assert np.linalg.norm(ref["Js"]) > 0
    cfg = wl.cfg
    grid, pals = dl.Grid.from_config(cfg), dl.Pals.from_config(cfg)
    _, D = dl.pals_field(grid, pals, torch.tensor(wl.theta_ref, device=dev), cfg.mus_prime)
    with dl.Operator(grid, D) as op:
        mua = op.pals_mua(pals, torch.tensor(th, device=dev)).cpu().numpy()
        assert np.max(np.abs(mua - prob.mua(wl.theta_ref))) <= 1e-13 * mua.max()
        U, Z = torch.tensor(ref["U"], device=dev), torch.tensor(ref["Z"], device=dev)
        Js = op.jacobian(U, Z, dl.DOT_JAC_FP64).cpu().numpy()
        g = op.grad_misfit(U, Z, torch.tensor(ref["Rs"], device=dev)).cpu().numpy()
    assert np.linalg.norm(Js - ref["Js"]) <= 1e-12 * np.linalg.norm(ref["Js"])
    assert np.linalg.norm(g - ref["g"]) <= 1e-12 * np.linalg.norm(ref["g"])
    # every RBF has nonzero columns (a lost band list would zero them)
    na = cfg.n_active_per_rbf
    for m in range(cfg.m0):
        assert np.linalg.norm(Js[:, m * na:(m + 1) * na]) > 0, m


@pytest.mark.parametrize("name", ["t3d_b", "t3d_c"])
def test_jacobian_and_gradient_bitwise_deterministic(dl, dev, name):
    wl = synthetic.make_workload(synthetic.get_config(name))
    op, W, V, rhs, res = gpu_fields(dl, dev, wl, wl.theta_ref, dl.DOT_FP64, 1e-12)
    ls = wl.cfg.l_s
    with op:
        U, Z = res.x[:, :ls], res.x[:, ls:]
        rng = np.random.default_rng(5)
        Rs = torch.tensor(rng.standard_normal((V.shape[1], ls)), device=dev)
        for prec in (dl.DOT_JAC_FP64, dl.DOT_JAC_SPLIT_BF16, dl.DOT_JAC_SPLIT_BF16X3):
            a = op.jacobian(U, Z, prec)
            b = op.jacobian(U, Z, prec)
            assert torch.equal(a, b), prec
        g1 = op.grad_misfit(U, Z, Rs)
        g2 = op.grad_misfit(U, Z, Rs)
        assert torch.equal(g1, g2)
