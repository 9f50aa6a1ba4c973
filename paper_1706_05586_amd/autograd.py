"""Differentiable sampled misfit f(p) = 1/2 ||V^T (C^T A(p)^{-1} B W - D W)||_F^2.

Section 3.1: with simultaneous sources W and detectors V the sampled misfit
needs l_s forward solves, and its gradient (eq. UnbiasedGrad) needs the
adjoint fields: g = J_s^T vec(R_s) = -G^T rowsum(U * (Z R_s)), where
Z = A^{-T} C V are the l_d adjoint fields and G = h^d d mu / d p.

``MisfitFn.apply(params, problem)`` runs, in the HIP library,
  forward : PaLS absorption at theta(params), B W and C V, the l_s + l_d
            solves in one multi-RHS call, the sampled residual and misfit;
  backward: the adjoint gradient kernel on the stored fields.
Modes:
  store_fields=True  (default) keeps U and Z from the forward pass
                     (checkpointed forward fields);
  store_fields=False keeps nothing large and re-solves in backward
                     (bitwise the same gradient: the solves are deterministic);
  adjoint_in_backward=True solves only U forward and, in backward, the l_s
                     adjoint systems A^T Lambda = C (V R_s) instead of Z.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L
from .api import Operator, Pals, empty_colmajor, gemm

__all__ = ["MisfitProblem", "MisfitFn", "misfit"]


@dataclass
class MisfitProblem:
    op: Operator
    pals: Pals
    theta: torch.Tensor           # (m0, 2 + d) template; active entries replaced by params
    src_cells: np.ndarray
    det_cells: np.ndarray
    W: torch.Tensor               # (n_s, l_s)
    V: torch.Tensor               # (n_d, l_d)
    DW: torch.Tensor              # (n_d, l_s) data times W
    rtol: float = 1e-12
    precision: int = L.DOT_FP64
    store_fields: bool = True
    adjoint_in_backward: bool = False

    def __post_init__(self):
        d = self.theta.shape[1] - 2
        cols = []
        if self.pals.active & L.DOT_ACT_ALPHA:
            cols.append(0)
        if self.pals.active & L.DOT_ACT_BETA:
            cols.append(1)
        if self.pals.active & L.DOT_ACT_CHI:
            cols += list(range(2, 2 + d))
        self._cols = torch.tensor(cols, device=self.theta.device)
        self._theta_key = None

    @property
    def n_p(self) -> int:
        return self.theta.shape[0] * len(self._cols)

    def params_of(self, theta: torch.Tensor) -> torch.Tensor:
        return theta[:, self._cols].reshape(-1).clone()

    def theta_of(self, params: torch.Tensor) -> torch.Tensor:
        th = self.theta.clone()
        th[:, self._cols] = params.detach().reshape(self.theta.shape[0], -1)
        return th

    def set_theta(self, theta: torch.Tensor):
        key = theta.detach().cpu().numpy().tobytes()
        if key != self._theta_key:
            self.op.pals_mua(self.pals, theta)
            self._theta_key = key

    def forward_fields(self, with_adjoint: bool):
        ls, ld = self.W.shape[1], self.V.shape[1]
        k = ls + ld if with_adjoint else ls
        rhs = empty_colmajor(self.op.N, k, self.W.device)
        self.op.form_rhs(self.src_cells, self.W, out=rhs[:, :ls])
        if with_adjoint:
            self.op.form_rhs(self.det_cells, self.V, out=rhs[:, ls:])
        res = self.op.solve(rhs, rtol=self.rtol, precision=self.precision)
        if not res.converged:
            raise RuntimeError(f"forward solve not converged: {res.relres.max():.3e}")
        return res.x[:, :ls], (res.x[:, ls:] if with_adjoint else None)


class MisfitFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, prob: MisfitProblem):
        theta = prob.theta_of(params)
        prob.set_theta(theta)
        with_adj = not prob.adjoint_in_backward
        U, Z = prob.forward_fields(with_adj)
        Rs, f = prob.op.sampled_misfit(prob.det_cells, U, prob.V, prob.DW)
        ctx.prob = prob
        ctx.theta = theta
        if prob.store_fields:
            ctx.fields = (U, Z)
        else:
            ctx.fields = None
        ctx.Rs = Rs
        return torch.tensor(f, dtype=torch.float64, device=params.device)

    @staticmethod
    def backward(ctx, grad_out):
        prob: MisfitProblem = ctx.prob
        prob.set_theta(ctx.theta)
        if ctx.fields is not None:
            U, Z = ctx.fields
        else:
            U, Z = prob.forward_fields(not prob.adjoint_in_backward)
        Rs = ctx.Rs
        if Z is not None:
            g = prob.op.grad_misfit(U, Z, Rs)
        else:
            # Lambda = A^{-T} C (V R_s): l_s adjoint solves, then the same
            # gradient kernel with R_s replaced by the identity
            VR = gemm(prob.V, Rs)
            rhs = prob.op.form_rhs(prob.det_cells, VR)
            res = prob.op.solve(rhs, rtol=prob.rtol, precision=prob.precision, trans=1)
            ls = U.shape[1]
            eye = torch.eye(ls, dtype=torch.float64, device=U.device)
            g = prob.op.grad_misfit(U, res.x, eye)
        return g * grad_out, None


def misfit(params: torch.Tensor, prob: MisfitProblem) -> torch.Tensor:
    return MisfitFn.apply(params, prob)
