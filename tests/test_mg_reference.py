"""Pins of the scipy model of the solver's multigrid V-cycle (the CG
preconditioner this build chose; tests/mg_reference.py) by properties a mistake in a transfer, a scaling or a smoothing
step breaks: symmetry and positive definiteness of the preconditioner, the
conditioning of the preconditioned operator, and the CG iteration count.
"""

import numpy as np
import pytest

from oracle import discretization as disc
import mg_reference as omg

ROBIN, DIRICHLET = 1, 0


def smooth_fields(n, seed):
    """A variable D and mu of the kind the PaLS phantoms give: smooth bumps."""
    rng = np.random.default_rng(seed)
    x = disc.cell_centres(n)
    mu = np.full(x.shape[0], 0.01)
    D = np.full(x.shape[0], 1.0 / 3.0)
    for _ in range(3):
        c = rng.uniform(0.2, 0.8, size=len(n)) * np.array(n) / n[0]
        r2 = np.sum((x - c) ** 2, axis=1)
        mu += 0.04 * np.exp(-r2 / 0.02)
        D *= 1.0 - 0.2 * np.exp(-r2 / 0.05)
    return D, mu


def test_level_shapes():
    assert omg.level_shapes((128, 128, 128)) == [(128,) * 3, (64,) * 3, (32,) * 3, (16,) * 3,
                                                 (8,) * 3, (4,) * 3]
    assert omg.level_shapes((96, 96, 96))[-1] == (3, 3, 3)
    assert omg.level_shapes((32, 16, 8)) == [(32, 16, 8), (16, 8, 4)]
    assert omg.level_shapes((19, 13, 11)) == [(19, 13, 11), (10, 7, 6), (5, 4, 3)]
    assert omg.level_shapes((70, 33, 17)) == [(70, 33, 17), (35, 17, 9), (18, 9, 5), (9, 5, 3)]
    assert omg.level_shapes((32, 32)) == [(32, 32), (16, 16), (8, 8), (4, 4)]
    assert omg.level_shapes((37, 29)) == [(37, 29), (19, 15), (10, 8), (5, 4)]
    assert omg.level_shapes((4, 40, 40)) == [(4, 40, 40)]


def test_transfers_ragged_aggregates():
    """P^T sums the children and P copies the parent, also where the last
    aggregate of an odd side holds fewer cells: P^T 1 counts the children."""
    for n, counts in (((5, 3), [4, 2, 2, 1]), ((3, 2, 3), [8, 4, 8, 4])):
        N = int(np.prod(n))
        cnt = omg._sum_children(np.ones(N), n)
        assert cnt.sum() == N
        # the corner aggregates at (0, 0, 0), (last x), (last y) and (last x, y)
        nc = [(v + 1) // 2 for v in n]
        corners = [0, nc[0] - 1, nc[0] * (nc[1] - 1), nc[0] * nc[1] - 1]
        assert list(cnt[corners]) == counts
        rng = np.random.default_rng(1)
        u, vc = rng.standard_normal(N), rng.standard_normal(cnt.size)
        # adjoint pair: <P^T u, vc> = <u, P vc>
        assert abs(omg._sum_children(u, n) @ vc - u @ omg._copy_to_children(vc, n)) <= 1e-13 * N


@pytest.fixture(scope="module")
def small():
    n = (8, 8, 8)
    bc = (DIRICHLET, DIRICHLET, DIRICHLET, ROBIN, ROBIN, ROBIN)
    D, mu = smooth_fields(n, 1)
    A = disc.assemble(n, bc, D, mu)
    lv = omg.hierarchy(n, bc, D, mu)
    M = omg.apply(lv, np.eye(A.shape[0]))
    return A.toarray(), M, lv


def test_preconditioner_symmetric_positive_definite(small):
    A, M, lv = small
    assert len(lv) == 2
    assert np.linalg.norm(M - M.T) <= 1e-13 * np.linalg.norm(M)
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    assert ev.min() > 0.0


def test_preconditioned_operator_well_conditioned(small):
    A, M, lv = small
    # eigenvalues of M A (similar to the symmetric L^T A L with M = L L^T)
    L = np.linalg.cholesky(0.5 * (M + M.T))
    ev = np.linalg.eigvalsh(L.T @ A @ L)
    d = np.sqrt(np.diag(A))
    evj = np.linalg.eigvalsh(A / np.outer(d, d))
    kappa_mg, kappa_j = ev.max() / ev.min(), evj.max() / evj.min()
    # the coarse correction removes the smooth modes Jacobi leaves behind
    assert kappa_mg < 0.1 * kappa_j, (kappa_mg, kappa_j)
    # symmetric smoothing with w < 1 on an operator with lambda_max(D^-1 A) <= 2:
    # M A has no eigenvalue beyond 2
    assert ev.max() < 2.0


def pcg(A, b, Minv, rtol, maxit=5000):
    x = np.zeros_like(b)
    r = b.copy()
    z = Minv(r)
    p = z.copy()
    rho = r @ z
    bn = np.linalg.norm(b)
    for it in range(1, maxit + 1):
        w = A @ p
        al = rho / (p @ w)
        x += al * p
        r -= al * w
        if np.linalg.norm(r) <= rtol * bn:
            return x, it
        z = Minv(r)
        rn = r @ z
        p = z + (rn / rho) * p
        rho = rn
    return x, maxit


def test_pcg_iterations_far_below_jacobi():
    n = (32, 32, 16)
    bc = (DIRICHLET, DIRICHLET, DIRICHLET, DIRICHLET, ROBIN, ROBIN)
    D, mu = smooth_fields(n, 2)
    A = disc.assemble(n, bc, D, mu)
    lv = omg.hierarchy(n, bc, D, mu)
    assert [l["n"] for l in lv] == [(32, 32, 16), (16, 16, 8), (8, 8, 4)]
    rng = np.random.default_rng(5)
    b = np.zeros(A.shape[0])
    b[rng.integers(0, A.shape[0], 20)] = rng.choice([-1.0, 1.0], 20)
    dg = A.diagonal()
    xj, itj = pcg(A, b, lambda r: r / dg, 1e-10)
    xm, itm = pcg(A, b, lambda r: omg.apply(lv, r), 1e-10)
    assert np.linalg.norm(b - A @ xm) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(xm - xj) <= 1e-8 * np.linalg.norm(xj)
    assert itm * 8 <= itj, (itm, itj)


def test_four_level_cycle_symmetric_positive():
    """On a grid with four levels (every smoothing count in use) the cycle is
    still symmetric and positive: u^T M v = v^T M u and v^T M v > 0 for
    random u, v."""
    n = (32, 32, 32)
    bc = (DIRICHLET, DIRICHLET, DIRICHLET, ROBIN, ROBIN, ROBIN)
    D, mu = smooth_fields(n, 3)
    lv = omg.hierarchy(n, bc, D, mu)
    assert len(lv) == 4
    rng = np.random.default_rng(9)
    u, v = rng.standard_normal((2, lv[0]["sd"].size))
    Mu, Mv = omg.apply(lv, u), omg.apply(lv, v)
    assert abs(u @ Mv - v @ Mu) <= 1e-13 * abs(u @ Mv)
    assert v @ Mv > 0.0 and u @ Mu > 0.0


@pytest.mark.parametrize("n", [(9, 7, 5), (11, 9)])
def test_ragged_and_2d_cycles_symmetric_positive_definite(n):
    """Odd sides (ragged last aggregates) and a 2D grid: the dense M is
    symmetric positive definite and M A has no eigenvalue beyond 2."""
    bc = (ROBIN, DIRICHLET, ROBIN, ROBIN, DIRICHLET, ROBIN)[:2 * len(n)]
    D, mu = smooth_fields(n, 4)
    A = disc.assemble(n, bc, D, mu).toarray()
    lv = omg.hierarchy(n, bc, D, mu)
    assert len(lv) >= 2
    M = omg.apply(lv, np.eye(A.shape[0]))
    assert np.linalg.norm(M - M.T) <= 1e-13 * np.linalg.norm(M)
    L = np.linalg.cholesky(0.5 * (M + M.T))
    ev = np.linalg.eigvalsh(L.T @ A @ L)
    assert ev.min() > 0.0 and ev.max() < 2.0


@pytest.mark.parametrize("n,factor", [((70, 33, 17), 8), ((37, 29), 8), ((101, 77), 16)])
def test_pcg_iterations_odd_and_2d_grids(n, factor):
    """On grids with odd sides, and in 2D, the cycle still takes CG to the
    tolerance in a fraction of Jacobi-PCG's iterations."""
    bc = (ROBIN, ROBIN, DIRICHLET, ROBIN, ROBIN, ROBIN)[:2 * len(n)]
    D, mu = smooth_fields(n, 6)
    A = disc.assemble(n, bc, D, mu)
    lv = omg.hierarchy(n, bc, D, mu)
    rng = np.random.default_rng(7)
    b = np.zeros(A.shape[0])
    b[rng.integers(0, A.shape[0], 12)] = rng.choice([-1.0, 1.0], 12)
    dg = A.diagonal()
    _, itj = pcg(A, b, lambda r: r / dg, 1e-10)
    xm, itm = pcg(A, b, lambda r: omg.apply(lv, r), 1e-10)
    assert np.linalg.norm(b - A @ xm) <= 1e-10 * np.linalg.norm(b)
    assert itm * factor <= itj, (itm, itj)
