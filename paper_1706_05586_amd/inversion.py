"""Outer inversion driver on the library (Sections 2, 3.2 and 4; tables T1, T3).

The paper's flow, every large step in the HIP library:
  1. sample average approximation (SAA): Gauss-Newton on the sampled problem
     min ||(W^T kron V^T)(r(p) + J d)|| (eq. TREGS J) with fixed random
     simultaneous sources W and detectors V, until the sampled misfit
     ||R_s||_F^2 reaches delta ||D||_F^2 (the intermediate tolerance);
  2. once: the full Jacobian J at that point (eq. Jtensor; n_s + n_d solves,
     the contraction run tile by tile), Alg. 1 for q_s optimized sources and
     q_d optimized detectors, and the complementary random samples
     (eqs. newW, newV), so W and V keep l_s and l_d columns;
  3. Gauss-Newton with the new W, V to ||R_s||^2 <= delta^2 ||D||^2
     (discrepancy principle).
Each phase is a trust-region Gauss-Newton method on the truncated SVD of the
sampled Jacobian J_s = L diag(s) R^T (the paper cites TREGS, which favours
the directions of the large singular values; its GCV-like rule is not
reproduced): with c = L^T vec(R_s) and the singular values above rcut s_1,
the step takes the leading terms -(c_i / s_i) R_i in full while they fit the
trust radius and the next one shortened by kappa to reach it.  A trial point
is accepted when f drops by more than eta times the model's reduction
sum_{full terms} c_i^2 / 2 + (kappa - kappa^2 / 2) c_t^2; the radius becomes
a quarter of the step after a ratio below 1/4 and at least twice the step
after one above 3/4.

Counting (the accounting of tables T1 and T3): per phase It trial steps,
FE = It + 1 function evaluations of l_s forward solves and JE Jacobian
evaluations of l_d adjoint solves; an optimized update adds n_s + n_d.
Every solve the driver runs is also counted as it is launched.

Host work is bookkeeping and the scalar decisions of the trust region on
small vectors copied back (singular values, c); fields, solves, misfits,
Jacobians, SVDs, steps and parameter updates run in the library.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from .api import (Operator, Pals, complemented_sample, empty_colmajor, gemm, optimized_design,
                  svd_thin, tsvd_step)

__all__ = ["TrustRegionOptions", "SampledDOT", "PhaseResult", "tr_gauss_newton", "invert",
           "solve_count", "sketched_design", "sketch_solves"]


@dataclass
class TrustRegionOptions:
    radius0: float = 1.0
    radius_max: float = 100.0
    eta: float = 1e-4
    rcut: float = 1e-4
    max_iter: int = 50
    pred_rtol: float = 1e-12   # stop when the model reduction is below this times f
    radius_min: float = 1e-12  # stop when a rejection shrinks the radius below this


@dataclass
class PhaseResult:
    p: torch.Tensor
    f: float
    radius: float
    it: int = 0
    fe: int = 0
    je: int = 0
    converged: bool = False
    history: list = field(default_factory=list)


def _step_choice(s: np.ndarray, c: np.ndarray, radius: float, rcut: float):
    """(t full terms, kappa of the shortened next term, step norm, model
    reduction) of the trust-region truncated-SVD step."""
    if s.size == 0 or not s[0] > 0:
        return 0, 0.0, 0.0, 0.0
    kept = int(np.count_nonzero(s > rcut * s[0]))
    coef = c[:kept] / s[:kept]
    sq = np.cumsum(coef * coef)
    t = int(np.count_nonzero(np.sqrt(sq) <= radius))
    full = float(sq[t - 1]) if t else 0.0
    kappa = 0.0
    red = 0.5 * float(np.sum(c[:t] * c[:t]))
    norm2 = full
    if t < kept:
        if coef[t] != 0:
            kappa = min(np.sqrt(max(radius * radius - full, 0.0)) / abs(coef[t]), 1.0)
        norm2 += (kappa * coef[t]) ** 2
        red += (kappa - 0.5 * kappa * kappa) * float(c[t] * c[t])
    return t, kappa, float(np.sqrt(norm2)), red


def _svd_factors(J: torch.Tensor, rcut: float):
    """J = Lf diag(s) Rf^T from the library's thin SVD of J or J^T."""
    rows, cols = J.shape
    if rows <= cols:
        s, Lf, Rf = svd_thin(J, rcut)
    else:
        s, Rf, Lf = svd_thin(J.t(), rcut)
    return s, Lf, Rf


def tr_gauss_newton(evaluate, jacobian, p0: torch.Tensor, f_stop: float,
                    opts: TrustRegionOptions, radius: float | None = None) -> PhaseResult:
    """One phase on the library: evaluate(p) -> (f, r (rows,), state) and
    jacobian(p, state) -> J_s (rows x n_p), both on the GPU."""
    radius = opts.radius0 if radius is None else radius
    p = p0.clone()
    f, r, state = evaluate(p)
    res = PhaseResult(p=p, f=f, radius=radius, fe=1)
    if f <= f_stop:
        res.converged = True
        return res
    J = jacobian(p, state)
    res.je = 1
    one = torch.ones((1, 1), dtype=torch.float64, device=p.device)
    while res.it < opts.max_iter:
        s, Lf, Rf = _svd_factors(J, opts.rcut)
        c = gemm(Lf, r.reshape(-1, 1), transa=True)
        t, kappa, step_norm, pred = _step_choice(s.cpu().numpy(), c.reshape(-1).cpu().numpy(),
                                                 radius, opts.rcut)
        if pred <= opts.pred_rtol * f:
            break                      # stationary: the model offers no reduction
        # p + d_t + kappa (d_{t+1} - d_t), d_k the step over k leading terms
        p_trial = empty_colmajor(p.numel(), 1, p.device)
        p_trial.copy_(p.reshape(-1, 1))
        if t > 0:
            d = tsvd_step(Lf, s, Rf, r, t)
            gemm(d.reshape(-1, 1), one, alpha=1.0 - kappa, beta=1.0, out=p_trial)
        if kappa > 0:
            d = tsvd_step(Lf, s, Rf, r, t + 1)
            gemm(d.reshape(-1, 1), one, alpha=kappa, beta=1.0, out=p_trial)
        p_trial = p_trial.reshape(-1)
        f_t, r_t, state_t = evaluate(p_trial)
        res.it += 1
        res.fe += 1
        ratio = (f - f_t) / pred
        accept = ratio > opts.eta
        if ratio < 0.25:
            radius = 0.25 * step_norm
        elif ratio > 0.75:
            radius = min(max(radius, 2.0 * step_norm), opts.radius_max)
        res.history.append(dict(t=t, kappa=kappa, step_norm=step_norm, pred=pred, f=f,
                                f_trial=f_t, ratio=ratio, accept=accept, radius=radius))
        if accept:
            p, f, r, state = p_trial, f_t, r_t, state_t
            if f <= f_stop:
                res.converged = True
                break
            J = jacobian(p, state)
            res.je += 1
        elif radius < opts.radius_min:
            break
    res.p, res.f, res.radius = p, f, radius
    return res


class SampledDOT:
    """r_s(p) = vec(V^T (C^T A(p)^-1 B W - D W)) and J_s on one operator.

    theta_template: (m0, 2 + d) parameters whose active entries the parameter
    vector p replaces (per RBF in the order alpha, beta, chi, as the
    Jacobian's columns).  data: (n_d, n_s) measurements."""

    def __init__(self, op: Operator, pals: Pals, theta_template: torch.Tensor, src_cells,
                 det_cells, data: torch.Tensor, rtol: float = 1e-10,
                 precision: int = L.DOT_FP64, jac_precision: int = L.DOT_JAC_FP64):
        self.op, self.pals = op, pals
        self.template = theta_template.clone()
        self.src_cells = np.asarray(src_cells, dtype=np.int32)
        self.det_cells = np.asarray(det_cells, dtype=np.int32)
        self.data = data
        self.rtol, self.precision, self.jac_precision = rtol, precision, jac_precision
        d = theta_template.shape[1] - 2
        cols = []
        if pals.active & L.DOT_ACT_ALPHA:
            cols.append(0)
        if pals.active & L.DOT_ACT_BETA:
            cols.append(1)
        if pals.active & L.DOT_ACT_CHI:
            cols += list(range(2, 2 + d))
        self._cols = torch.tensor(cols, device=theta_template.device)
        self._key = None
        self.solves = 0

    def params_of(self, theta: torch.Tensor) -> torch.Tensor:
        return theta[:, self._cols].reshape(-1).contiguous()

    def theta_of(self, p: torch.Tensor) -> torch.Tensor:
        th = self.template.clone()
        th[:, self._cols] = p.reshape(th.shape[0], -1)
        return th

    def _set(self, p: torch.Tensor):
        th = self.theta_of(p)
        key = th.cpu().numpy().tobytes()
        if key != self._key:
            self.op.pals_mua(self.pals, th)
            self._key = key

    def set_samples(self, W: torch.Tensor, V: torch.Tensor):
        self.W, self.V = W, V
        self.DW = gemm(self.data, W)

    def _solve(self, rhs: torch.Tensor, trans: int = 0) -> torch.Tensor:
        res = self.op.solve(rhs, rtol=self.rtol, precision=self.precision, trans=trans)
        if not res.converged:
            raise RuntimeError(f"solve did not converge: relres {res.relres.max():.3e}")
        self.solves += rhs.shape[1]
        return res.x

    def evaluate(self, p: torch.Tensor):
        self._set(p)
        U = self._solve(self.op.form_rhs(self.src_cells, self.W))
        Rs, f = self.op.sampled_misfit(self.det_cells, U, self.V, self.DW)
        # vec(R_s): the column-major storage of R_s read in order
        r = Rs.t().reshape(-1)
        return f, r, U

    def jacobian(self, p: torch.Tensor, U: torch.Tensor) -> torch.Tensor:
        self._set(p)
        Z = self._solve(self.op.form_rhs(self.det_cells, self.V), trans=1)
        return self.op.jacobian(U, Z, self.jac_precision)

    def full_jacobian(self, p: torch.Tensor) -> torch.Tensor:
        """J of eq. Jtensor: the fields of every source and every detector."""
        self._set(p)
        dev = self.data.device
        n_s, n_d = len(self.src_cells), len(self.det_cells)
        U = self._solve(self.op.form_rhs(self.src_cells,
                                         torch.eye(n_s, dtype=torch.float64, device=dev)))
        Z = self._solve(self.op.form_rhs(self.det_cells,
                                         torch.eye(n_d, dtype=torch.float64, device=dev)),
                        trans=1)
        return self.op.jacobian(U, Z, self.jac_precision)


def solve_count(phases, l_s: int, l_d: int, n_updates: int, n_s: int, n_d: int,
                update_solves: int | None = None) -> int:
    """FE l_s + JE l_d per phase plus, per optimized update, n_s + n_d (full
    Jacobian) or update_solves (sketched design)."""
    per_update = n_s + n_d if update_solves is None else update_solves
    return sum(ph.fe * l_s + ph.je * l_d for ph in phases) + n_updates * per_update


# ------------------------------------------------------------ sketched design
# Alg. 1 without the full Jacobian (Section 3.2's remark on a randomized
# low-rank approximation; Section 5).  The unfoldings J~, K~, L~ of the
# Jacobian tensor (entries c_m^T A^-1 dA/dp_k A^-1 b_j, written without the
# minus sign as in Alg. 1) are sketched with Khatri-Rao test vectors
# x kron theta, theta over the parameters: E[omega omega^T] = I, so Y Y^T / k
# estimates each unfolding's Gram without bias, and the leading left singular
# vectors of Y replace those of the unfolding.  A test vector costs one
# forward and one adjoint solve:
#   J~ (w kron theta) = C^T A^-1 (dA/d theta) A^-1 B w
#   K~ (a kron theta) = B^T A^-T (dA/d theta) A^-T C V~ a
#   L~ (a kron theta) = C^T A^-1 (dA/d theta) A^-1 B W~ a.
# Step (1) once, steps (2)-(3) for a fixed number of sweeps with fresh test
# vectors.

def sketch_solves(k: int, sweeps: int) -> int:
    return 2 * k * (1 + 2 * sweeps)


def _readout(op: Operator, cells, S: torch.Tensor) -> torch.Tensor:
    """S at the given cells (n x k): the misfit kernel with V = I and no data."""
    n, k = len(cells), S.shape[1]
    eye = torch.eye(n, dtype=torch.float64, device=S.device)
    zero = torch.zeros((n, k), dtype=torch.float64, device=S.device)
    R, _ = op.sampled_misfit(cells, S, eye, zero)
    return R


def _leading(Y: torch.Tensor, q: int) -> torch.Tensor:
    """Leading q left singular vectors of Y (n x k) from the library's SVD."""
    n, k = Y.shape
    if k <= n:
        _, _, Lv = svd_thin(Y.t(), 1e-12)
    else:
        _, Lv, _ = svd_thin(Y, 1e-12)
    return Lv[:, :q]


def sketched_design(sdot: "SampledDOT", p: torch.Tensor, q_s: int, q_d: int, draws: dict,
                    y_signs: torch.Tensor, z_signs: torch.Tensor):
    """Optimized and complementary samples from the sketched Alg. 1 at p.
    draws (device tensors): w1 (n_s x k), t1 (n_p x k), lists a2, t2, a3, t3
    per sweep.  Returns (W, V, info) with the sketches, the directions after
    each sketch (V_init, then W_s and V_s per sweep) and the solve count."""
    sdot._set(p)
    op = sdot.op
    before = sdot.solves

    def det_side(X, Th):            # C^T A^-1 (dA/d theta) A^-1 B X
        F = sdot._solve(op.form_rhs(sdot.src_cells, X))
        return _readout(op, sdot.det_cells, sdot._solve(op.dadp_apply(Th, F), trans=1))

    def src_side(Yd, Th):           # B^T A^-T (dA/d theta) A^-T C Yd
        F = sdot._solve(op.form_rhs(sdot.det_cells, Yd), trans=1)
        return _readout(op, sdot.src_cells, sdot._solve(op.dadp_apply(Th, F)))

    sk = {"Y1": det_side(draws["w1"], draws["t1"])}
    V = _leading(sk["Y1"], q_d)
    dirs = {"V_init": V}
    W = None
    for s in range(len(draws["a2"])):
        sk[f"Y2_{s}"] = src_side(gemm(V, draws["a2"][s]), draws["t2"][s])
        W = _leading(sk[f"Y2_{s}"], q_s)
        sk[f"Y3_{s}"] = det_side(gemm(W, draws["a3"][s]), draws["t3"][s])
        V = _leading(sk[f"Y3_{s}"], q_d)
        dirs[f"W_{s}"], dirs[f"V_{s}"] = W, V
    Wn = complemented_sample(W, y_signs)
    Vn = complemented_sample(V, z_signs)
    return Wn, Vn, {"sketches": sk, "directions": dirs, "W_tilde": W, "V_tilde": V,
                    "solves": sdot.solves - before}


def invert(sdot: SampledDOT, p0: torch.Tensor, W0: torch.Tensor, V0: torch.Tensor, q_s: int,
           q_d: int, y_signs: torch.Tensor, z_signs: torch.Tensor, delta: float,
           opts: TrustRegionOptions, final_tol: float | None = None,
           hooi_tol: float = 1e-10, hooi_maxit: int = 50, sketch: dict | None = None):
    """SAA phase to the intermediate tolerance delta, one optimized update (Alg. 1
    on the full Jacobian, or the sketched design when the test vectors
    `sketch` are given), then Gauss-Newton to final_tol (default delta^2)."""
    final_tol = delta * delta if final_tol is None else final_tol
    dflat = sdot.data.t().reshape(-1, 1) if sdot.data.t().is_contiguous() else \
        sdot.data.reshape(-1, 1)
    dnorm2 = float(gemm(dflat, dflat, transa=True).item())      # ||D||_F^2
    n_s, l_s = W0.shape
    n_d, l_d = V0.shape
    sdot.set_samples(W0, V0)
    saa = tr_gauss_newton(sdot.evaluate, sdot.jacobian, p0, 0.5 * delta * dnorm2, opts)
    phases, n_up = [saa], 0
    out = dict(saa=saa, p_saa=saa.p.clone())
    update_solves = None
    if (q_s > 0 or q_d > 0) and sketch is None:
        J = sdot.full_jacobian(saa.p)
        n_up = 1
        dev = J.device
        I_s = torch.eye(n_s, dtype=torch.float64, device=dev)
        I_d = torch.eye(n_d, dtype=torch.float64, device=dev)
        W, V, info = optimized_design(J, I_s, I_d, q_s, q_d, y_signs, z_signs, hooi_tol,
                                      hooi_maxit)
        out.update(J_full=J, W=W, V=V, W_opt=W[:, :q_s], V_opt=V[:, :q_d],
                   hooi_iters=info["hooi_iters"], hooi_objective=info["objective"])
    elif q_s > 0 or q_d > 0:
        n_up = 1
        W, V, info = sketched_design(sdot, saa.p, q_s, q_d, sketch, y_signs, z_signs)
        update_solves = info["solves"]
        out.update(W=W, V=V, W_opt=W[:, :q_s], V_opt=V[:, :q_d], sketches=info["sketches"])
    if q_s > 0 or q_d > 0:
        sdot.set_samples(W, V)
        opt = tr_gauss_newton(sdot.evaluate, sdot.jacobian, saa.p, 0.5 * final_tol * dnorm2,
                              opts, radius=saa.radius)
        phases.append(opt)
        out["opt"] = opt
    out["p"] = phases[-1].p
    out["solves"] = solve_count(phases, l_s, l_d, n_up, n_s, n_d, update_solves)
    out["counted"] = sdot.solves
    return out
