"""Thin Python layer over the dotpath C ABI.

Matrices are passed as torch tensors with their logical (rows, cols) shape;
the ABI wants column-major device memory, which is what ``A.t().contiguous()``
holds, so a field block U of logical shape (N, l) lives in memory as a
contiguous (l, N) tensor and is returned as its transposed view.  torch
supplies device memory and the current stream only: every arithmetic step
runs in the HIP kernels of libdotpath.so.
"""

from __future__ import annotations

import ctypes as C
import warnings
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L
from ._lib import check, lib

__all__ = ["Grid", "Pals", "Operator", "SolveResult", "pals_field", "gemm", "colmajor",
           "check_field_block",
           "empty_colmajor", "mode_gram", "symeig", "qr_complete", "hooi", "svd_thin",
           "tsvd_step", "optimized_design", "complemented_sample"]


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _need_cuda_f64(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")


def colmajor(t: torch.Tensor, name: str = "array") -> torch.Tensor:
    """Memory of a logical (rows, cols) matrix in column-major order: a contiguous
    (cols, rows) tensor (no copy when t already is such a transposed view)."""
    _need_cuda_f64(t, name)
    if t.dim() == 1:
        return t.contiguous()
    return t.t().contiguous()


def empty_colmajor(rows: int, cols: int, device) -> torch.Tensor:
    """Storage for a column-major (rows, cols) matrix; returns the (rows, cols) view."""
    return torch.empty((cols, rows), dtype=torch.float64, device=device).t()


def _workspace(nbytes: int, device) -> torch.Tensor:
    w = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    off = (-w.data_ptr()) % 256
    return w[off:off + max(int(nbytes), 256)]


@dataclass(frozen=True)
class Grid:
    dim: int
    n: tuple
    bc: tuple

    def c(self) -> L.DotGrid:
        g = L.DotGrid()
        g.dim = self.dim
        n = list(self.n) + [1] * (3 - len(self.n))
        for a in range(3):
            g.n[a] = int(n[a])
        bc = list(self.bc) + [0] * (6 - len(self.bc))
        for f in range(6):
            g.bc[f] = int(bc[f])
        return g

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    @classmethod
    def from_config(cls, cfg) -> "Grid":
        return cls(dim=cfg.dim, n=tuple(cfg.n), bc=tuple(cfg.bc[: 2 * cfg.dim]))


@dataclass(frozen=True)
class Pals:
    m0: int
    active: int
    mu_in: float
    mu_out: float
    cutoff: float
    eps: float
    gamma: float

    def c(self) -> L.DotPals:
        p = L.DotPals()
        p.m0, p.active = int(self.m0), int(self.active)
        p.mu_in, p.mu_out, p.cutoff, p.eps, p.gamma = (self.mu_in, self.mu_out, self.cutoff,
                                                       self.eps, self.gamma)
        return p

    @classmethod
    def from_config(cls, cfg) -> "Pals":
        return cls(m0=cfg.m0, active=cfg.active, mu_in=cfg.mu_in, mu_out=cfg.mu_out,
                   cutoff=cfg.cutoff, eps=cfg.eps, gamma=cfg.gamma)

    def n_act(self, dim: int) -> int:
        return ((self.active & 1) > 0) + ((self.active & 2) > 0) + (dim if self.active & 4 else 0)


def pals_field(grid: Grid, pals: Pals, theta: torch.Tensor, mus_prime: float | None = None):
    """mu(x_c; theta) on the grid, and D = 1/(3 (mu + mus')) when mus_prime is given."""
    _need_cuda_f64(theta, "theta")
    theta = theta.contiguous()
    mua = torch.empty(grid.N, dtype=torch.float64, device=theta.device)
    diff = torch.empty_like(mua) if mus_prime is not None else None
    g, p = grid.c(), pals.c()
    check(lib.dot_pals_field(C.byref(g), C.byref(p), _ptr(theta),
                             float(mus_prime or 0.0), _ptr(mua),
                             _ptr(diff) if diff is not None else None, _stream()),
          "dot_pals_field")
    return (mua, diff) if diff is not None else mua


def check_field_block(t: torch.Tensor, rows: int, cols: int, name: str = "out"):
    """A caller-supplied (rows, cols) block that the library writes whole: float64,
    on the GPU, column-major with leading dimension rows (t.t() contiguous)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if tuple(t.shape) != (rows, cols):
        raise ValueError(f"{name} must have shape ({rows}, {cols}), got {tuple(t.shape)}")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {t.dtype}")
    if not t.t().is_contiguous():
        raise ValueError(f"{name} must be column-major: {name}.t() contiguous")
    if not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")


def _check_colmajor_out(out: torch.Tensor, rows: int, cols: int):
    if out.shape != (rows, cols) or out.dtype != torch.float64 or not out.is_cuda:
        raise ValueError(f"out must be a float64 CUDA ({rows}, {cols}) matrix")
    if cols > 1 and out.stride() != (1, rows) and not (out.stride(0) == 1 and out.stride(1) >= rows):
        raise ValueError("out must be column-major")


def gemm(A: torch.Tensor, B: torch.Tensor, transa: bool = False, transb: bool = False,
         alpha: float = 1.0, out: torch.Tensor | None = None, beta: float = 0.0) -> torch.Tensor:
    """alpha op(A) op(B) + beta out for logical matrices, computed by the library's
    FP64 kernel.  ``out`` may be a column block of a column-major matrix; it is
    required when beta is not zero."""
    Am, Bm = colmajor(A, "A"), colmajor(B, "B")
    ar, ac = A.shape
    br, bc = B.shape
    m, kd = (ac, ar) if transa else (ar, ac)
    kb, n = (bc, br) if transb else (br, bc)
    if kd != kb:
        raise ValueError("inner dimensions differ")
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs out")
        out = empty_colmajor(m, n, A.device)
        ldc = max(m, 1)
    else:
        _check_colmajor_out(out, m, n)
        ldc = out.stride(1) if n > 1 else max(m, 1)
    check(lib.dot_gemm(int(transa), int(transb), m, n, kd, float(alpha), _ptr(Am), max(ar, 1),
                       _ptr(Bm), max(br, 1), float(beta), _ptr(out), ldc, _stream()), "dot_gemm")
    return out


def mode_gram(T: torch.Tensor, dims, mode: int) -> torch.Tensor:
    """Gram matrix of the mode-0 or mode-1 unfolding of a column-major 3-tensor
    (flat float64 CUDA tensor of dims[0] * dims[1] * dims[2] values)."""
    dA, dB, dC = (int(v) for v in dims)
    _need_cuda_f64(T, "T")
    if T.numel() != dA * dB * dC or not T.is_contiguous():
        raise ValueError("T must hold dA*dB*dC contiguous values")
    R = dA if mode == 0 else dB
    G = empty_colmajor(R, R, T.device)
    nb = int(lib.dot_mode_gram_workspace_bytes(dA, dB, dC, mode))
    w = _workspace(nb, T.device)
    check(lib.dot_mode_gram(dA, dB, dC, _ptr(T), mode, _ptr(G), _ptr(w), w.numel(), _stream()),
          "dot_mode_gram")
    return G


def symeig(A: torch.Tensor):
    """Eigenvalues (descending) and eigenvectors of a symmetric matrix (cyclic Jacobi)."""
    n = A.shape[0]
    Am = colmajor(A, "A")
    w = torch.empty(n, dtype=torch.float64, device=A.device)
    V = empty_colmajor(n, n, A.device)
    nb = int(lib.dot_symeig_workspace_bytes(n))
    work = _workspace(nb, A.device)
    sweeps = C.c_int(0)
    check(lib.dot_symeig(n, _ptr(Am), n, _ptr(w), _ptr(V), n, _ptr(work), work.numel(),
                         C.byref(sweeps), _stream()), "dot_symeig")
    return w, V


def qr_complete(X: torch.Tensor) -> torch.Tensor:
    """Complete orthogonal factor Q (n x n) of X (n x q): Q[:, :q] spans range(X)."""
    n, q = X.shape
    Xm = colmajor(X, "X")
    Q = empty_colmajor(n, n, X.device)
    w = _workspace(int(lib.dot_qr_workspace_bytes(n, q)), X.device)
    check(lib.dot_qr_complete(n, q, _ptr(Xm), n, _ptr(Q), n, _ptr(w), w.numel(), _stream()),
          "dot_qr_complete")
    return Q


def hooi(J: torch.Tensor, n_d: int, n_s: int, q_d: int, q_s: int, tol: float = 1e-10,
         maxit: int = 50):
    """Alg. 1 on the (n_d n_s) x n_p Jacobian (detector index fastest).
    Returns (W~ (n_s x q_s), V~ (n_d x q_d), iterations, objective)."""
    Jm = colmajor(J, "J")
    n_p = J.shape[1]
    if J.shape[0] != n_d * n_s:
        raise ValueError("J must have n_d * n_s rows")
    W = empty_colmajor(n_s, q_s, J.device)
    V = empty_colmajor(n_d, q_d, J.device)
    nb = int(lib.dot_hooi_workspace_bytes(n_d, n_s, n_p, q_d, q_s))
    work = _workspace(nb, J.device)
    it, obj = C.c_int(0), C.c_double(0.0)
    check(lib.dot_hooi(n_d, n_s, n_p, _ptr(Jm), q_d, q_s, float(tol), int(maxit), _ptr(W),
                       _ptr(V), C.byref(it), C.byref(obj), _ptr(work), work.numel(), _stream()),
          "dot_hooi")
    return W, V, it.value, obj.value


def svd_thin(A: torch.Tensor, rcut: float = 1e-12):
    """Thin SVD of an m x n matrix (m <= n): (s, U, Y) with A = U diag(s) Y^T."""
    m, n = A.shape
    Am = colmajor(A, "A")
    s = torch.empty(m, dtype=torch.float64, device=A.device)
    U = empty_colmajor(m, m, A.device)
    Y = empty_colmajor(n, m, A.device)
    work = _workspace(int(lib.dot_svd_workspace_bytes(m, n)), A.device)
    check(lib.dot_svd_thin(m, n, _ptr(Am), m, _ptr(s), _ptr(U), m, _ptr(Y), n, float(rcut),
                           _ptr(work), work.numel(), _stream()), "dot_svd_thin")
    return s, U, Y


def tsvd_step(L: torch.Tensor, s: torch.Tensor, R: torch.Tensor, r: torch.Tensor, t: int):
    """Truncated-SVD Gauss-Newton step for min ||J d + r|| with J = L diag(s) R^T:
    d = -sum_{i < t} (L[:, i]^T r / s_i) R[:, i]."""
    rows, k = L.shape
    cols = R.shape[0]
    if R.shape[1] != k or s.numel() < k or r.numel() != rows:
        raise ValueError("shape mismatch in tsvd_step")
    Lm, Rm = colmajor(L, "L"), colmajor(R, "R")
    _need_cuda_f64(s, "s")
    _need_cuda_f64(r, "r")
    x = torch.empty(cols, dtype=torch.float64, device=L.device)
    work = _workspace(int(lib.dot_tsvd_step_workspace_bytes(int(t))), L.device)
    check(lib.dot_tsvd_step(rows, cols, k, _ptr(Lm), rows, _ptr(s.contiguous()), _ptr(Rm), cols,
                            int(t), _ptr(r.contiguous()), _ptr(x), _ptr(work), work.numel(),
                            _stream()), "dot_tsvd_step")
    return x


def optimized_design(Js: torch.Tensor, W: torch.Tensor, V: torch.Tensor, q_s: int, q_d: int,
                     y_signs: torch.Tensor, z_signs: torch.Tensor, tol: float = 1e-10,
                     maxit: int = 50):
    """Optimized and complementary simultaneous sources/detectors (Section 3.2).

    Alg. 1 on the sampled Jacobian J_s gives W~ (l_s x q_s) and V~ (l_d x q_d);
    the optimized directions are lifted to the full spaces as W_hat =
    orth(W W~), V_hat = orth(V V~) by Householder QR, whose complete Q also
    gives the complements W_c, V_c; the new samples are W = [W_hat, W_c Y]
    and V = [V_hat, V_c Z] with Y = (l_s - q_s)^{-1/2} y_signs (eqs. newW, newV).
    The new samples have q + (columns of the signs) columns each; with W and V
    identities, J_s is the full Jacobian and the design is the paper's.
    Returns (W_new, V_new, info)."""
    n_s, l_s = W.shape
    n_d, l_d = V.shape
    Wt, Vt, it, obj = hooi(Js, l_d, l_s, q_d, q_s, tol, maxit)
    Wn = complemented_sample(gemm(W, Wt), y_signs)
    Vn = complemented_sample(gemm(V, Vt), z_signs)
    return Wn, Vn, {"hooi_iters": it, "objective": obj, "W_tilde": Wt, "V_tilde": Vt}


def complemented_sample(X: torch.Tensor, signs: torch.Tensor) -> torch.Tensor:
    """New simultaneous sources (or detectors) from optimized directions
    (eqs. newW, newV): X (n x q) spans them; Householder QR gives the complete
    Q = [X_hat, X_c]; returns [X_hat, X_c Y], Y = signs / sqrt(l - q), signs
    (n - q) x (l - q)."""
    n, q = X.shape
    if signs.shape[0] != n - q:
        raise ValueError(f"complement signs must have {n - q} rows")
    l = q + signs.shape[1]
    Q = qr_complete(X)
    new = empty_colmajor(n, l, X.device)
    new[:, :q].copy_(Q[:, :q])
    if l > q:
        gemm(Q[:, q:], signs, alpha=1.0 / np.sqrt(l - q), out=new[:, q:])
    return new


@dataclass
class SolveResult:
    x: torch.Tensor          # logical (N, k) view of column-major storage
    iters: np.ndarray        # per column
    relres: np.ndarray       # true ||b - A x|| / ||b|| per column (binary64)
    iters_max: int
    outer: int
    converged: bool


class Operator:
    """Handle over dot_op: A(p) on one grid, owned device arrays freed on close()."""

    def __init__(self, grid: Grid, D: torch.Tensor):
        _need_cuda_f64(D, "D")
        if D.numel() != grid.N:
            raise ValueError("D must have one value per cell")
        self.grid = grid
        self.device = D.device
        self._handle = C.c_void_p()
        g = grid.c()
        check(lib.dot_build_operator(C.byref(g), _ptr(D.contiguous()), _stream(),
                                     C.byref(self._handle)), "dot_build_operator")
        self.pals = None

    # ------------------------------------------------------------ lifetime
    def close(self):
        if self._handle:
            lib.dot_destroy_operator(self._handle)
            self._handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def N(self) -> int:
        return self.grid.N

    # ------------------------------------------------------------ operator
    def set_mua(self, mua: torch.Tensor):
        _need_cuda_f64(mua, "mua")
        check(lib.dot_set_mua(self._handle, _ptr(mua.contiguous()), _stream()), "dot_set_mua")
        self.pals = None

    def pals_mua(self, pals: Pals, theta: torch.Tensor) -> torch.Tensor:
        _need_cuda_f64(theta, "theta")
        mua = torch.empty(self.N, dtype=torch.float64, device=self.device)
        p = pals.c()
        check(lib.dot_pals_mua(self._handle, C.byref(p), _ptr(theta.contiguous()), _ptr(mua),
                               _stream()), "dot_pals_mua")
        self.pals = pals
        return mua

    def pals_mua_diffusion(self, pals: Pals, theta: torch.Tensor, mus_in: float,
                           mus_out: float):
        """A(theta) with mu and D = 1 / (3 (mu + mu_s)) both from the level set
        (diffusion inverted as well).  Returns (mu, D)."""
        _need_cuda_f64(theta, "theta")
        mua = torch.empty(self.N, dtype=torch.float64, device=self.device)
        D = torch.empty_like(mua)
        p = pals.c()
        check(lib.dot_pals_mua_diffusion(self._handle, C.byref(p), float(mus_in), float(mus_out),
                                         _ptr(theta.contiguous()), _ptr(mua), _ptr(D), _stream()),
              "dot_pals_mua_diffusion")
        self.pals = pals
        return mua, D

    @property
    def n_pairs(self) -> int:
        """(RBF, cell) pairs of the band lists of the last pals_mua call."""
        return int(lib.dot_pals_pairs(self._handle))

    @property
    def n_band_cells(self) -> int:
        """Distinct cells of those band lists (rows of U and Z the contraction reads)."""
        return int(lib.dot_pals_band_cells(self._handle))

    @property
    def multigrid_levels(self) -> int:
        """Levels of the V-cycle hierarchy the solver uses (0: Jacobi)."""
        return int(lib.dot_multigrid_levels(self._handle))

    def multigrid_cycle_bytes(self, precision: int) -> float:
        """Algorithmic HBM bytes per column of one V-cycle (0: no hierarchy)."""
        return float(lib.dot_multigrid_cycle_bytes(self._handle, int(precision)))

    def multigrid_apply(self, R: torch.Tensor) -> torch.Tensor:
        """One binary64 V-cycle as an approximate inverse of A (N x k in and out)."""
        Rm = colmajor(R, "R")
        k = R.shape[1]
        Z = empty_colmajor(self.N, k, self.device)
        nbytes = int(lib.dot_multigrid_workspace_bytes(self._handle, k))
        work = _workspace(max(nbytes, 256), self.device)
        check(lib.dot_multigrid_apply(self._handle, k, _ptr(Rm), _ptr(Z), _ptr(work), work.numel(),
                                      _stream()), "dot_multigrid_apply")
        return Z

    def apply(self, X: torch.Tensor) -> torch.Tensor:
        X2 = X.reshape(-1, 1) if X.dim() == 1 else X
        Xm = colmajor(X2, "X")
        k = X2.shape[1]
        Y = empty_colmajor(self.N, k, self.device)
        check(lib.dot_apply(self._handle, k, _ptr(Xm), _ptr(Y), _stream()), "dot_apply")
        return Y.reshape(-1) if X.dim() == 1 else Y

    def form_rhs(self, cells, weights: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """B W: weights is (n_pts, k); returns the (N, k) right-hand side block.
        ``out`` may be a column slice of a larger column-major block."""
        cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int32))
        Wm = colmajor(weights, "weights")
        n_pts, k = weights.shape
        if cells.size != n_pts:
            raise ValueError("one cell per weight row")
        if out is not None:
            check_field_block(out, self.N, k)
            rhs = out
        else:
            rhs = empty_colmajor(self.N, k, self.device)
        check(lib.dot_form_rhs(self._handle, n_pts, cells.ctypes.data_as(L._pi32), k, _ptr(Wm),
                               _ptr(rhs), _stream()), "dot_form_rhs")
        return rhs

    def solve_workspace_bytes(self, k: int, precision: int) -> int:
        return int(lib.dot_solve_workspace_bytes(self._handle, k, precision))

    def solve(self, rhs: torch.Tensor, rtol: float = 1e-10, precision: int = L.DOT_FP64,
              max_iter: int = 20000, inner_rtol: float = 0.1,
              check_every: int = 8, trans: int = 0, out: torch.Tensor | None = None,
              work: torch.Tensor | None = None, warn: bool = True,
              precond: int = L.DOT_PRECOND_AUTO) -> SolveResult:
        Bm = colmajor(rhs, "rhs")
        k = rhs.shape[1]
        if rhs.shape[0] != self.N:
            raise ValueError(f"rhs must have {self.N} rows")
        if out is not None:
            check_field_block(out, self.N, k)
        x = out if out is not None else empty_colmajor(self.N, k, self.device)
        nbytes = self.solve_workspace_bytes(k, precision)
        if work is None or work.numel() < nbytes or work.data_ptr() % 256:
            work = _workspace(nbytes, self.device)
        opts = L.DotSolveOpts(rtol, max_iter, precision, inner_rtol, check_every, precond)
        iters = np.zeros(k, dtype=np.int32)
        rel = np.zeros(k, dtype=np.float64)
        info = L.DotSolveInfo(0, 0, iters.ctypes.data_as(C.POINTER(C.c_int32)),
                              rel.ctypes.data_as(C.POINTER(C.c_double)))
        code = lib.dot_solve_multi_rhs(self._handle, trans, k, _ptr(Bm), _ptr(x), C.byref(opts),
                                       _ptr(work), work.numel(), C.byref(info), _stream())
        check(code, "dot_solve_multi_rhs")
        if code == L.DOT_NOT_CONVERGED and warn:
            warnings.warn(f"solve did not reach rtol={rtol}: max relres {rel.max():.3e}",
                          L.NotConverged)
        return SolveResult(x=x, iters=iters, relres=rel, iters_max=info.iters_max,
                           outer=info.outer, converged=code == L.DOT_OK)

    def solve_complex(self, rhs: torch.Tensor, kappa: float, rtol: float = 1e-10,
                      max_iter: int = 20000, check_every: int = 8,
                      precond: int = L.DOT_PRECOND_AUTO, warn: bool = True,
                      precision: int = L.DOT_FP64) -> SolveResult:
        """(A + i kappa h^d I) X = rhs for a complex128 (N, k) block (COCG).
        precision DOT_MIXED runs the V-cycle preconditioner in binary32 (COCG
        stays binary64).  The result's x is complex128 (N, k)."""
        if not isinstance(rhs, torch.Tensor) or rhs.dtype != torch.complex128 or not rhs.is_cuda:
            raise TypeError("rhs must be a complex128 CUDA tensor")
        R2 = rhs.reshape(-1, 1) if rhs.dim() == 1 else rhs
        if R2.shape[0] != self.N:
            raise ValueError(f"rhs must have {self.N} rows")
        k = R2.shape[1]
        # N x 2k real block: real parts, then imaginary parts (column-major)
        B = empty_colmajor(self.N, 2 * k, self.device)
        B[:, :k].copy_(R2.real)
        B[:, k:].copy_(R2.imag)
        X = empty_colmajor(self.N, 2 * k, self.device)
        nbytes = int(lib.dot_solve_complex_workspace_bytes(self._handle, k, precond))
        work = _workspace(nbytes, self.device)
        opts = L.DotSolveOpts(rtol, max_iter, precision, 0.1, check_every, precond)
        iters = np.zeros(k, dtype=np.int32)
        rel = np.zeros(k, dtype=np.float64)
        info = L.DotSolveInfo(0, 0, iters.ctypes.data_as(C.POINTER(C.c_int32)),
                              rel.ctypes.data_as(C.POINTER(C.c_double)))
        code = lib.dot_solve_complex(self._handle, float(kappa), k, _ptr(B), _ptr(X),
                                     C.byref(opts), _ptr(work), work.numel(), C.byref(info),
                                     _stream())
        check(code, "dot_solve_complex")
        if code == L.DOT_NOT_CONVERGED and warn:
            warnings.warn(f"complex solve did not reach rtol={rtol}: max relres {rel.max():.3e}",
                          L.NotConverged)
        x = torch.complex(X[:, :k], X[:, k:])
        return SolveResult(x=x.reshape(-1) if rhs.dim() == 1 else x, iters=iters, relres=rel,
                           iters_max=info.iters_max, outer=0, converged=code == L.DOT_OK)

    # ------------------------------------------------------------ profiling
    def profile_enable(self, on: bool = True):
        check(lib.dot_profile_enable(self._handle, int(on)), "dot_profile_enable")

    def profile_kinds(self, *kinds: int):
        """Time only these DOT_PROF_* kinds (profile_enable selects all)."""
        mask = 0
        for k in kinds:
            mask |= 1 << int(k)
        check(lib.dot_profile_kinds(self._handle, mask), "dot_profile_kinds")

    def profile_read(self, kind: int):
        """(summed event ms, launches, sum over launches of active columns)."""
        ms, n, cols = C.c_double(), C.c_int64(), C.c_int64()
        check(lib.dot_profile_read(self._handle, kind, C.byref(ms), C.byref(n), C.byref(cols)),
              "dot_profile_read")
        return ms.value, n.value, cols.value

    # ------------------------------------------------------------ estimators
    def sampled_misfit(self, det_cells, U: torch.Tensor, V: torch.Tensor, DW: torch.Tensor):
        """R_s = V^T (C^T U - D W) and f = 1/2 ||R_s||_F^2."""
        det = np.ascontiguousarray(np.asarray(det_cells, dtype=np.int32))
        Um, Vm, DWm = colmajor(U, "U"), colmajor(V, "V"), colmajor(DW, "DW")
        n_d, l_d = V.shape
        l_s = U.shape[1]
        if DW.shape != (n_d, l_s) or det.size != n_d:
            raise ValueError("shape mismatch in sampled_misfit")
        Rs = empty_colmajor(l_d, l_s, self.device)
        f = C.c_double(0.0)
        check(lib.dot_sampled_misfit(self._handle, n_d, det.ctypes.data_as(L._pi32), l_s, _ptr(Um),
                                     l_d, _ptr(Vm), _ptr(DWm), _ptr(Rs), C.byref(f), _stream()),
              "dot_sampled_misfit")
        return Rs, f.value

    def jacobian_workspace_bytes(self, l_s: int, l_d: int) -> int:
        return int(lib.dot_jacobian_workspace_bytes(self._handle, l_s, l_d))

    def jacobian(self, U: torch.Tensor, Z: torch.Tensor, precision: int = L.DOT_JAC_FP64,
                 work: torch.Tensor | None = None) -> torch.Tensor:
        if self.pals is None:
            raise RuntimeError("call pals_mua before jacobian")
        Um, Zm = colmajor(U, "U"), colmajor(Z, "Z")
        l_s, l_d = U.shape[1], Z.shape[1]
        n_p = self.pals.m0 * self.pals.n_act(self.grid.dim)
        Js = empty_colmajor(l_s * l_d, n_p, self.device)
        nbytes = self.jacobian_workspace_bytes(l_s, l_d)
        if work is None or work.numel() < nbytes or work.data_ptr() % 256:
            work = _workspace(nbytes, self.device)
        check(lib.dot_jacobian(self._handle, l_s, _ptr(Um), l_d, _ptr(Zm), precision, _ptr(Js),
                               _ptr(work), work.numel(), _stream()), "dot_jacobian")
        return Js

    def dadp_apply(self, Theta: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
        """(sum_k Theta[k, j] dA/dp_k) X[:, j] for each column j (Theta: n_p x k)."""
        if self.pals is None:
            raise RuntimeError("call pals_mua before dadp_apply")
        n_p = self.pals.m0 * self.pals.n_act(self.grid.dim)
        Th2 = Theta.reshape(-1, 1) if Theta.dim() == 1 else Theta
        X2 = X.reshape(-1, 1) if X.dim() == 1 else X
        if Th2.shape[0] != n_p or X2.shape != (self.N, Th2.shape[1]):
            raise ValueError(f"Theta must be ({n_p}, k) and X ({self.N}, k)")
        Tm, Xm = colmajor(Th2, "Theta"), colmajor(X2, "X")
        k = X2.shape[1]
        Y = empty_colmajor(self.N, k, self.device)
        check(lib.dot_dadp_apply(self._handle, k, _ptr(Tm), _ptr(Xm), _ptr(Y), _stream()),
              "dot_dadp_apply")
        return Y.reshape(-1) if X.dim() == 1 else Y

    def grad_misfit(self, U: torch.Tensor, Z: torch.Tensor, Rs: torch.Tensor,
                    work: torch.Tensor | None = None) -> torch.Tensor:
        if self.pals is None:
            raise RuntimeError("call pals_mua before grad_misfit")
        Um, Zm, Rm = colmajor(U, "U"), colmajor(Z, "Z"), colmajor(Rs, "Rs")
        l_s, l_d = U.shape[1], Z.shape[1]
        n_p = self.pals.m0 * self.pals.n_act(self.grid.dim)
        g = torch.empty(n_p, dtype=torch.float64, device=self.device)
        nbytes = self.jacobian_workspace_bytes(l_s, l_d)
        if work is None or work.numel() < nbytes or work.data_ptr() % 256:
            work = _workspace(nbytes, self.device)
        check(lib.dot_grad_misfit(self._handle, l_s, _ptr(Um), l_d, _ptr(Zm), _ptr(Rm), _ptr(g),
                                  _ptr(work), work.numel(), _stream()), "dot_grad_misfit")
        return g

    def grad_misfit_noalloc(self, U: torch.Tensor, Z: torch.Tensor, Rs: torch.Tensor,
                            out: torch.Tensor) -> torch.Tensor:
        """grad_misfit through the library's allocation-free entry point: the
        caller supplies ``out`` (n_p float64 values), U, Z and Rs already
        column-major (as the solver returns them), and the library uses its
        fixed per-GPU scratch array."""
        if self.pals is None:
            raise RuntimeError("call pals_mua before grad_misfit_noalloc")
        l_s, l_d = U.shape[1], Z.shape[1]
        n_p = self.pals.m0 * self.pals.n_act(self.grid.dim)
        for t, name, rows, cols in ((U, "U", self.N, l_s), (Z, "Z", self.N, l_d),
                                    (Rs, "Rs", l_d, l_s)):
            check_field_block(t, rows, cols, name)
        if (not isinstance(out, torch.Tensor) or out.dtype != torch.float64 or not out.is_cuda
                or out.numel() != n_p or not out.is_contiguous()):
            raise ValueError(f"out must be a contiguous float64 CUDA tensor of {n_p} values")
        check(lib.dot_grad_misfit_noalloc(self._handle, l_s, _ptr(U), l_d, _ptr(Z), _ptr(Rs),
                                          _ptr(out), _stream()), "dot_grad_misfit_noalloc")
        return out
