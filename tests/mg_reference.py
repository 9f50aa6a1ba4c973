"""Reference model of the solver's multigrid preconditioner (test support).

This is not part of the oracle: the paper leaves the iterative solver open
(Section 3.3: iterative or sparse direct solvers), so nothing here is the
paper's arithmetic.  It is a plain scipy model of the geometric multigrid
V-cycle that this build chose as the preconditioner of its CG, written so
that the GPU V-cycle can be compared with it element by element and so that
the design itself (symmetry, definiteness, its effect on CG) can be pinned
on the CPU.  The solves themselves are checked against the oracle by other
means: residuals recomputed with the oracle's CSR matrix and the forward
error against its direct solve.

The design, written out:

  * levels: level l + 1 aggregates the 2 x 2 x 2 cells of level l, while
    all three sides are even and the smallest is at least 8; every level is
    the finite-volume operator of `oracle.discretization.assemble` on its own
    grid, with D and mu the means over the children (so the coarse mass is
    the sum of the fine masses);
  * each level in the symmetrically scaled form A^_l = S_l^-1 A_l S_l^-1,
    S_l = diag(A_l)^(1/2);
  * transfers with the piecewise-constant prolongation P (a coarse value
    copied to its 8 children), in scaled variables
        prolongation  x^_l += S_l P S_{l+1}^-1 x^_{l+1}
        restriction   b^_{l+1} = S_{l+1}^-1 P^T S_l r^_l
  * one cycle on level l with right-hand side b, J(v) = v + w (b - A^ v)
    the damped Jacobi step and nu = NU0 on level 0, NU1 on level 1, NU2
    below:
        x = J applied nu - 1 times to w b;
        b_{l+1} = restriction of (b - A^ x);  x_{l+1} = cycle(b_{l+1});
        result: J applied nu times to x + prolongation of x_{l+1}
    and on the coarsest level NU_C steps J from x = 0, with w = OMEGA;
  * as an approximate inverse of A: M R = S_0^-1 V(S_0^-1 R).

Pinned (tests/test_mg_reference.py) by properties a mistake in a transfer, a
scaling or the smoothing would break: M is symmetric and positive definite
(dense on a small grid), M A has a condition number far below that of the
Jacobi-scaled A, and CG preconditioned with M needs a fraction of the
iterations of Jacobi-PCG.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from oracle import discretization as disc

OMEGA = 0.85
NU0 = 2
NU1 = 3
NU2 = 5
NU_C = 8


def level_shapes(n) -> list:
    """Cells per axis (n_x, n_y, n_z) of each level; a single level in 2D or
    when the grid does not halve."""
    n = tuple(int(v) for v in n)
    out = [n]
    if len(n) != 3:
        return out
    while all(v % 2 == 0 for v in n) and min(n) >= 8:
        n = tuple(v // 2 for v in n)
        out.append(n)
    return out


def _coarsen_mean(a: np.ndarray) -> np.ndarray:
    z, y, x = a.shape
    return a.reshape(z // 2, 2, y // 2, 2, x // 2, 2).mean(axis=(1, 3, 5))


def hierarchy(n, bc, D: np.ndarray, mua: np.ndarray) -> list:
    """Per level: cells per axis, the scaled operator A^ (CSR) and S = sqrt(diag A)."""
    shapes = level_shapes(n)
    Dl = np.asarray(D, dtype=np.float64).reshape(shapes[0][::-1])
    ml = np.asarray(mua, dtype=np.float64).reshape(shapes[0][::-1])
    levels = []
    for li, nl in enumerate(shapes):
        if li > 0:
            Dl, ml = _coarsen_mean(Dl), _coarsen_mean(ml)
        A = disc.assemble(nl, bc, Dl.ravel(), ml.ravel())
        sd = np.sqrt(A.diagonal())
        Ah = sp.diags(1.0 / sd) @ A @ sp.diags(1.0 / sd)
        levels.append(dict(n=nl, A=A, Ah=sp.csr_matrix(Ah), sd=sd))
    return levels


def _sum_children(v: np.ndarray, n) -> np.ndarray:
    nx, ny, nz = n
    return v.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).sum(axis=(1, 3, 5)).ravel()


def _copy_to_children(vc: np.ndarray, n) -> np.ndarray:
    nx, ny, nz = n
    c = vc.reshape(nz // 2, ny // 2, nx // 2)
    return np.repeat(np.repeat(np.repeat(c, 2, axis=0), 2, axis=1), 2, axis=2).ravel()


def vcycle_scaled(levels: list, b: np.ndarray, level: int = 0) -> np.ndarray:
    """One V-cycle on the scaled system of `level` for one right-hand side."""
    L = levels[level]
    Ah = L["Ah"]
    if level == len(levels) - 1:
        x = OMEGA * b
        for _ in range(NU_C - 1):
            x = x + OMEGA * (b - Ah @ x)
        return x
    C = levels[level + 1]
    nu = NU0 if level == 0 else (NU1 if level == 1 else NU2)
    x = OMEGA * b
    for _ in range(nu - 1):
        x = x + OMEGA * (b - Ah @ x)
    bc = _sum_children(L["sd"] * (b - Ah @ x), L["n"]) / C["sd"]
    xc = vcycle_scaled(levels, bc, level + 1)
    y = x + L["sd"] * _copy_to_children(xc / C["sd"], L["n"])
    for _ in range(nu):
        y = y + OMEGA * (b - Ah @ y)
    return y


def apply(levels: list, R: np.ndarray) -> np.ndarray:
    """M R = S^-1 V(S^-1 R), column by column (R: N or N x k)."""
    R = np.asarray(R, dtype=np.float64)
    sd = levels[0]["sd"]
    if R.ndim == 1:
        return vcycle_scaled(levels, R / sd) / sd
    return np.stack([vcycle_scaled(levels, R[:, j] / sd) / sd for j in range(R.shape[1])], axis=1)
