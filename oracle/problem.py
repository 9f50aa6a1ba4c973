"""Oracle end-to-end evaluation of one workload (test infrastructure only).

Builds, from the seeded synthetic inputs: the frozen diffusion field from the
reference absorption, A(theta), the simultaneous source/detector matrices,
synthetic noisy data from theta_true, the forward/adjoint fields, the sampled
misfit, the sampled Jacobian and the gradient.  Every step calls the plain
functions of the sibling modules.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import discretization as disc
from . import estimators as est
from . import pals, solvers


@dataclass
class OracleProblem:
    n: tuple
    bc: tuple
    d: int
    h: float
    x: np.ndarray            # cell centres (N, d)
    D: np.ndarray            # frozen diffusion (N,)
    consts: dict             # mu_in, mu_out, cutoff, eps, gamma
    active: int

    @property
    def N(self) -> int:
        return self.x.shape[0]

    def mua(self, theta: np.ndarray) -> np.ndarray:
        return pals.mua(self.x, theta, **self.consts)

    def operator(self, theta: np.ndarray):
        return disc.assemble(self.n, self.bc, self.D, self.mua(theta))

    def G(self, theta: np.ndarray) -> np.ndarray:
        """h^d d mu / d p: column k is the diagonal of dA/dp_k."""
        return self.h ** self.d * pals.dmua_dp(self.x, theta, self.active, **self.consts)


def build(wl) -> OracleProblem:
    cfg = wl.cfg
    n = tuple(cfg.n)
    x = disc.cell_centres(n)
    consts = dict(mu_in=cfg.mu_in, mu_out=cfg.mu_out, cutoff=cfg.cutoff, eps=cfg.eps,
                  gamma=cfg.gamma)
    mua_ref = pals.mua(x, wl.theta_ref, **consts)
    D = disc.diffusion_from_mua(mua_ref, cfg.mus_prime)
    return OracleProblem(n=n, bc=tuple(cfg.bc[: 2 * cfg.dim]), d=cfg.dim, h=disc.spacing(n), x=x,
                         D=D, consts=consts, active=cfg.active)


def synthetic_data(prob: OracleProblem, wl) -> np.ndarray:
    """D_data = C^T A(theta_true)^{-1} B with 0.1% relative noise."""
    A_true = prob.operator(wl.theta_true)
    M = est.measurements(A_true, prob.n, wl.src_cells, wl.det_cells)
    return est.noisy_data(M, wl.xi, wl.cfg.noise)


def evaluate(prob: OracleProblem, wl, theta: np.ndarray, W: np.ndarray, V: np.ndarray,
             data: np.ndarray, with_jacobian: bool = True):
    """Fields, sampled residual, misfit, Jacobian and gradient at theta."""
    A = prob.operator(theta)
    BW = est.simultaneous_rhs(prob.N, wl.src_cells, W)
    CV = est.simultaneous_rhs(prob.N, wl.det_cells, V)
    U = solvers.direct_solve(A, BW, prob.n)
    Z = solvers.direct_solve(A.T.tocsr(), CV, prob.n)
    Rs = est.sampled_residual(U, wl.det_cells, V, data @ W)
    out = dict(A=A, BW=BW, CV=CV, U=U, Z=Z, Rs=Rs, f=est.misfit(Rs))
    if with_jacobian:
        G = prob.G(theta)
        out["G"] = G
        out["Js"] = est.jacobian_sparse_loops(U, Z, G)
        out["g"] = est.gradient_adjoint(U, Z, Rs, G)
    return out
