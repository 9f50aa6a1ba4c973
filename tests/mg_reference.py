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

  * levels: level l + 1 aggregates the 2 x 2 x 2 cells of level l (2 x 2
    in 2D; the last aggregate of an odd side is one cell thick along it),
    every side halved rounding up while each coarse side keeps at least 3
    cells; every level is the finite-volume operator of
    `oracle.discretization.assemble` on its own grid (h = 1 / n_x), with D
    and mu the means over the children (so a full aggregate's mass is the
    sum of its children's masses);
  * each level in the symmetrically scaled form A^_l = S_l^-1 A_l S_l^-1,
    S_l = diag(A_l)^(1/2);
  * transfers with the piecewise-constant prolongation P (a coarse value
    copied to its children), in scaled variables
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


MIN_SIDE = 3


def level_shapes(n) -> list:
    """Cells per axis of each level: every side halved, rounding up, while
    every coarse side keeps at least MIN_SIDE cells (2D grids stay 2D)."""
    n = tuple(int(v) for v in n)
    out = [n]
    while all((v + 1) // 2 >= MIN_SIDE for v in n):
        n = tuple((v + 1) // 2 for v in n)
        out.append(n)
    return out


def _parents(n) -> np.ndarray:
    """Coarse index of every fine cell (cell order i + n_x (j + n_y k))."""
    nc = [(v + 1) // 2 for v in n]
    idx = np.indices(tuple(reversed(n)))[::-1]        # x, y, (z) index arrays
    P = np.zeros(idx[0].shape, dtype=np.int64)
    stride = 1
    for a in range(len(n)):
        P += (idx[a] // 2) * stride
        stride *= nc[a]
    return P.ravel()


def _coarsen_mean(a: np.ndarray, n) -> np.ndarray:
    """Means over the children of each aggregate (fewer at an odd side's end)."""
    P = _parents(n)
    Nc = int(np.prod([(v + 1) // 2 for v in n]))
    return np.bincount(P, weights=a.ravel(), minlength=Nc) / np.bincount(P, minlength=Nc)


def hierarchy(n, bc, D: np.ndarray, mua: np.ndarray) -> list:
    """Per level: cells per axis, the scaled operator A^ (CSR) and S = sqrt(diag A)."""
    shapes = level_shapes(n)
    Dl = np.asarray(D, dtype=np.float64).ravel()
    ml = np.asarray(mua, dtype=np.float64).ravel()
    levels = []
    for li, nl in enumerate(shapes):
        if li > 0:
            Dl, ml = _coarsen_mean(Dl, shapes[li - 1]), _coarsen_mean(ml, shapes[li - 1])
        A = disc.assemble(nl, bc, Dl, ml)
        sd = np.sqrt(A.diagonal())
        Ah = sp.diags(1.0 / sd) @ A @ sp.diags(1.0 / sd)
        levels.append(dict(n=nl, A=A, Ah=sp.csr_matrix(Ah), sd=sd))
    return levels


def _sum_children(v: np.ndarray, n) -> np.ndarray:
    Nc = int(np.prod([(a + 1) // 2 for a in n]))
    return np.bincount(_parents(n), weights=v, minlength=Nc)


def _copy_to_children(vc: np.ndarray, n) -> np.ndarray:
    return vc[_parents(n)]


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
