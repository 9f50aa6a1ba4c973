"""Outer inversion driver (Sections 2, 3.2 and 4; tables T1 and T3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's flow: Gauss-Newton on the sampled problem (eq. TREGS J) with a
fixed set of random simultaneous sources W and detectors V (sample average
approximation, SAA) until the misfit reaches an intermediate tolerance; then,
once, the full Jacobian J (eq. Jtensor: n_s + n_d solves), Alg. 1 for q_s
optimized sources and q_d optimized detectors, the complementary random
samples (eqs. newW, newV), and Gauss-Newton with the new W, V to the final
tolerance (discrepancy principle).

Readings (the paper cites TREGS for the nonlinear solver and does not define
it; its GCV-like rule is not reproduced):
  * Each phase is a trust-region Gauss-Newton method on the truncated SVD of
    J_s = L diag(s) R^T (eqs. GN, Eq:NLLS): with c = L^T r and the singular
    values kept above rcut s_1, the step takes the leading terms
    -(c_i / s_i) R_i in full while they fit the trust radius and the next
    one shortened to reach it (the step moves continuously with the radius
    from the first singular direction towards the least-squares step), so
    the directions of the large singular values come first, as the paper
    describes for TREGS.
  * The Gauss-Newton model reduction of such a step is
    sum_{full terms} c_i^2 / 2 + (kappa - kappa^2 / 2) c_t^2, kappa the
    shortening of the partial term.  A trial point is
    accepted when the actual reduction of f = 1/2 ||r||^2 is more than eta
    times the model's; the radius shrinks to a quarter of the step after a
    ratio below 1/4 and grows to at least twice the step after a ratio above
    3/4 (capped at radius_max).
  * A phase also ends at a stationary point (model reduction below 1e-12 f)
    or when rejections shrink the radius below 1e-12.
  * Tolerances (Section 4): the misfit is measured as ||R_s||_F^2 / ||D||_F^2
    (the noise of relative level delta has squared norm about delta^2 ||D||^2);
    the intermediate tolerance is delta and the final one delta^2, both on
    the sampled estimate, which is what the method sees.
  * Counting (tables T1, T3): per phase, It trial steps, FE = It + 1 function
    evaluations (l_s forward solves each: the start and every trial point)
    and JE Jacobian evaluations (l_d adjoint solves each, at the start and
    at every accepted point from which the iteration continues); an
    optimized update adds n_s + n_d solves.  With these counts the table
    rows reproduce as FE l + JE l (+ n_s + n_d + the SAA phase's solves).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import design
from . import estimators as est
from . import randomized, solvers


@dataclass
class TrustRegionOptions:
    radius0: float = 1.0       # initial trust radius (parameter units)
    radius_max: float = 100.0
    eta: float = 1e-4          # acceptance threshold on the reduction ratio
    rcut: float = 1e-4         # singular values below rcut * s_1 are not used
    max_iter: int = 50         # trial steps per phase
    pred_rtol: float = 1e-12   # stop when the model reduction is below this times f
    radius_min: float = 1e-12  # stop when a rejection shrinks the radius below this


def truncated_step_coefficients(s: np.ndarray, c: np.ndarray, radius: float, rcut: float):
    """Terms of the trust-region truncated-SVD step.

    s: singular values (descending), c = L^T r.  With a_i = c_i / s_i over the
    kept singular values, the step is d = -sum_{i<t} a_i R_i - kappa a_t R_t:
    the t leading terms that fit the radius in full and, if more are kept,
    the next one shortened (0 <= kappa < 1) so that ||d|| reaches the radius.
    Returns (t, kappa, ||d||, predicted reduction of the Gauss-Newton model
    sum_{i<t} c_i^2 / 2 + (kappa - kappa^2 / 2) c_t^2)."""
    s = np.asarray(s, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    kept = int(np.sum(s > rcut * s[0])) if s.size and s[0] > 0 else 0
    if kept == 0:
        return 0, 0.0, 0.0, 0.0
    a = c[:kept] / s[:kept]
    sq = np.cumsum(a * a)
    t = int(np.sum(np.sqrt(sq) <= radius))
    full = float(sq[t - 1]) if t > 0 else 0.0
    kappa = 0.0
    if t < kept and a[t] != 0:
        kappa = min(np.sqrt(max(radius * radius - full, 0.0)) / abs(a[t]), 1.0)
    step_norm = float(np.sqrt(full + (kappa * a[t]) ** 2)) if t < kept else float(np.sqrt(full))
    pred = 0.5 * float(np.sum(c[:t] ** 2))
    if t < kept:
        pred += (kappa - 0.5 * kappa * kappa) * float(c[t] ** 2)
    return t, kappa, step_norm, pred


@dataclass
class PhaseResult:
    p: np.ndarray
    f: float
    radius: float
    it: int = 0
    fe: int = 0
    je: int = 0
    converged: bool = False
    history: list = field(default_factory=list)   # one dict per trial step


def tr_gauss_newton(evaluate, jacobian, p0: np.ndarray, f_stop: float,
                    opts: TrustRegionOptions, radius: float | None = None) -> PhaseResult:
    """One phase of trust-region Gauss-Newton on r(p).

    evaluate(p) -> (f, r, state) with f = 1/2 ||r||^2; jacobian(p, state) -> J.
    Stops when f <= f_stop, or after opts.max_iter trial steps."""
    radius = opts.radius0 if radius is None else radius
    p = np.array(p0, dtype=np.float64)
    f, r, state = evaluate(p)
    res = PhaseResult(p=p, f=f, radius=radius, fe=1)
    if f <= f_stop:
        res.converged = True
        return res
    J = jacobian(p, state)
    res.je = 1
    while res.it < opts.max_iter:
        Lm, s, Rt = np.linalg.svd(J, full_matrices=False)
        c = Lm.T @ r
        t, kappa, step_norm, pred = truncated_step_coefficients(s, c, radius, opts.rcut)
        if pred <= opts.pred_rtol * f:
            break                      # stationary: the model offers no reduction
        d = -(Rt[:t].T @ (c[:t] / s[:t]))
        if kappa > 0:
            d = d - kappa * (c[t] / s[t]) * Rt[t]
        p_trial = p + d
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


# ---------------------------------------------------------------- DOT problem

def params_of(theta: np.ndarray, active: int) -> np.ndarray:
    """Active parameters in the Jacobian's column order: per RBF, alpha, beta, chi."""
    return np.asarray(theta)[:, _active_cols(theta, active)].reshape(-1)


def theta_of(template: np.ndarray, p: np.ndarray, active: int) -> np.ndarray:
    th = np.array(template, dtype=np.float64)
    cols = _active_cols(th, active)
    th[:, cols] = np.asarray(p).reshape(th.shape[0], len(cols))
    return th


def _active_cols(theta, active):
    d = np.asarray(theta).shape[1] - 2
    cols = []
    if active & 1:
        cols.append(0)
    if active & 2:
        cols.append(1)
    if active & 4:
        cols += list(range(2, 2 + d))
    return cols


class SampledDOT:
    """The sampled residual r_s(p) = vec(V^T (C^T A(p)^-1 B W - D W)) and its
    Jacobian J_s (eqs. EsTResidual, Jacobian kth column) on an oracle problem,
    with every solve counted."""

    def __init__(self, prob, wl, data: np.ndarray, theta_template: np.ndarray):
        self.prob, self.wl, self.data = prob, wl, np.asarray(data)
        self.template = np.array(theta_template, dtype=np.float64)
        self.active = prob.active
        self.solves = 0

    def set_samples(self, W: np.ndarray, V: np.ndarray):
        self.W, self.V = np.asarray(W), np.asarray(V)
        self.DW = self.data @ self.W

    def evaluate(self, p):
        th = theta_of(self.template, p, self.active)
        A = self.prob.operator(th)
        BW = est.simultaneous_rhs(self.prob.N, self.wl.src_cells, self.W)
        U = solvers.direct_solve(A, BW, self.prob.n)
        self.solves += self.W.shape[1]
        Rs = est.sampled_residual(U, self.wl.det_cells, self.V, self.DW)
        return est.misfit(Rs), Rs.reshape(-1, order="F"), (th, A, U)

    def jacobian(self, p, state):
        th, A, U = state
        CV = est.simultaneous_rhs(self.prob.N, self.wl.det_cells, self.V)
        Z = solvers.direct_solve(A.T.tocsr(), CV, self.prob.n)
        self.solves += self.V.shape[1]
        return est.jacobian_sparse_loops(U, Z, self.prob.G(th))

    def full_jacobian(self, p):
        """J of eq. Jtensor (W = I, V = I): n_s + n_d solves."""
        th = theta_of(self.template, p, self.active)
        A = self.prob.operator(th)
        n_s, n_d = len(self.wl.src_cells), len(self.wl.det_cells)
        U = solvers.direct_solve(A, est.simultaneous_rhs(self.prob.N, self.wl.src_cells,
                                                         np.eye(n_s)), self.prob.n)
        Z = solvers.direct_solve(A.T.tocsr(), est.simultaneous_rhs(self.prob.N, self.wl.det_cells,
                                                                   np.eye(n_d)), self.prob.n)
        self.solves += n_s + n_d
        return est.jacobian_sparse_loops(U, Z, self.prob.G(th))

    def true_misfit(self, p) -> float:
        """||C^T A(p)^-1 B - D||_F^2 (not counted: a check on the side)."""
        th = theta_of(self.template, p, self.active)
        M = est.measurements(self.prob.operator(th), self.prob.n, self.wl.src_cells,
                             self.wl.det_cells)
        return float(np.sum((M - self.data) ** 2))


def solve_count(phases, l_s: int, l_d: int, n_updates: int, n_s: int, n_d: int,
                update_solves: int | None = None) -> int:
    """Large solves of a run: FE l_s + JE l_d per phase plus, per optimized
    update, n_s + n_d for the full Jacobian (the accounting of tables T1 and
    T3) or update_solves for a sketched design."""
    per_update = n_s + n_d if update_solves is None else update_solves
    return sum(ph.fe * l_s + ph.je * l_d for ph in phases) + n_updates * per_update


def invert(sdot: SampledDOT, p0: np.ndarray, W0: np.ndarray, V0: np.ndarray, q_s: int, q_d: int,
           y_signs: np.ndarray, z_signs: np.ndarray, delta: float,
           opts: TrustRegionOptions, final_tol: float | None = None, hooi_tol: float = 1e-10,
           hooi_maxit: int = 50, sketch: dict | None = None):
    """SAA phase to ||R_s||^2 <= delta ||D||^2, one optimized update, then
    Gauss-Newton to final_tol (default delta^2).  The update runs Alg. 1 on
    the full Jacobian, or, given the test vectors `sketch` (see
    randomized.randomized_hooi), the sketched Alg. 1 without it."""
    final_tol = delta * delta if final_tol is None else final_tol
    dnorm2 = float(np.sum(sdot.data ** 2))
    l_s, l_d = W0.shape[1], V0.shape[1]
    n_s, n_d = W0.shape[0], V0.shape[0]
    sdot.set_samples(W0, V0)
    saa = tr_gauss_newton(sdot.evaluate, sdot.jacobian, p0, 0.5 * delta * dnorm2, opts)
    phases, n_up = [saa], 0
    out = dict(saa=saa, p_saa=saa.p.copy())
    update_solves = None
    if q_s > 0 or q_d > 0:
        J = sdot.full_jacobian(saa.p)
        n_up = 1
        if sketch is None:
            Wt, Vt, hist, it = design.hooi(J, n_d, n_s, q_d, q_s, hooi_tol, hooi_maxit)
            out.update(hooi_iters=it, hooi_objective=hist[-1])
        else:
            # the sketches are contractions of J here (their definition); the
            # method itself forms them with two solves per test vector
            sdot.solves -= n_s + n_d
            Wt, Vt, sk = randomized.randomized_hooi(J, n_d, n_s, q_d, q_s, sketch)
            k, sweeps = sketch["w1"].shape[1], len(sketch["a2"])
            update_solves = randomized.sketch_solves(k, sweeps)
            sdot.solves += update_solves
            out.update(sketches=sk, hooi_objective=design.objective(J, Wt, Vt))
        Wc = design.orthonormal_complement(Wt)
        Vc = design.orthonormal_complement(Vt)
        W = design.complemented_sample(Wt, Wc, y_signs)
        V = design.complemented_sample(Vt, Vc, z_signs)
        out.update(J_full=J, W_opt=Wt, V_opt=Vt, W=W, V=V)
        sdot.set_samples(W, V)
        opt = tr_gauss_newton(sdot.evaluate, sdot.jacobian, saa.p, 0.5 * final_tol * dnorm2,
                              opts, radius=saa.radius)
        phases.append(opt)
        out["opt"] = opt
    out["p"] = phases[-1].p
    out["solves"] = solve_count(phases, l_s, l_d, n_up, n_s, n_d, update_solves)
    out["counted"] = sdot.solves
    return out
