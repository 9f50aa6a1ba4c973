"""Pins for the oracle's finite-volume operator (Section 2, eq. PDE).

* exact symmetry (A = A^T, so the adjoint solves reuse A);
* constant coefficients with Dirichlet faces: the discrete operator is
  diagonalized by the DST-II (ghost-cell odd reflection), so scipy's DST
  gives the exact discrete solution independently of the assembly code;
* Robin faces: a manufactured eigenfunction of the continuous Robin problem
  (cos(k (z - L/2)) with tan(k L / 2) = 1 / (2 D k)) converges at O(h^2),
  which a wrong Robin coefficient would break.
"""

import numpy as np
import pytest
import scipy.fft as sfft
import scipy.optimize as sopt

from oracle import discretization as disc
from oracle import solvers


def _rand_field(n, seed, lo=0.2, hi=0.5):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=disc.cell_shape(n))


@pytest.mark.parametrize("n,bc", [((9, 7), (1, 1, 0, 1)), ((6, 5, 4), (0, 0, 0, 0, 1, 1)),
                                  ((5, 7, 6), (1, 0, 0, 1, 1, 0))])
def test_symmetric_positive_definite(n, bc):
    D = _rand_field(n, 1)
    mu = _rand_field(n, 2, 0.0, 0.1)
    A = disc.assemble(n, bc, D, mu)
    assert abs(A - A.T).max() == 0.0
    w = np.linalg.eigvalsh(A.toarray())
    assert w.min() > 0.0
    # weak diagonal dominance with strict dominance on boundary rows
    Ad = A.toarray()
    off = np.abs(Ad).sum(axis=1) - np.abs(np.diag(Ad))
    assert np.all(np.diag(Ad) >= off - 1e-15)


def _dst_solve(n, Dc, mu, rhs):
    """Exact discrete solve for constant D, mu with all-Dirichlet faces via DST-II."""
    d = len(n)
    h = 1.0 / n[0]
    shape = disc.cell_shape(n)
    lam = np.zeros(shape)
    for a in range(d):
        k = np.arange(1, n[a] + 1)
        l1 = 2.0 - 2.0 * np.cos(np.pi * k / n[a])
        sh = [1] * d
        sh[d - 1 - a] = n[a]
        lam = lam + l1.reshape(sh)
    lam = h ** (d - 2) * Dc * lam + h ** d * mu
    bt = sfft.dstn(rhs.reshape(shape), type=2, norm="ortho")
    return sfft.idstn(bt / lam, type=2, norm="ortho").ravel()


@pytest.mark.parametrize("n", [(13, 9), (7, 5, 6), (8, 8, 8)])
def test_dirichlet_constant_coefficients_match_dst(n):
    d = len(n)
    N = int(np.prod(n))
    Dc, mu = 0.31, 0.04
    A = disc.assemble(n, (0,) * (2 * d), np.full(N, Dc), np.full(N, mu))
    rng = np.random.default_rng(3)
    b = rng.standard_normal(N)
    x_ref = _dst_solve(n, Dc, mu, b)
    x = solvers.splu_solve(A, b)
    assert np.linalg.norm(x - x_ref) <= 1e-12 * np.linalg.norm(x_ref)


def _robin_k(D, L):
    f = lambda k: 0.25 * np.cos(k * L / 2) - 0.5 * D * k * np.sin(k * L / 2)
    return sopt.brentq(f, 1e-9, np.pi / L - 1e-12)


def _manufactured_error_3d(nn, D, mu):
    n = (nn, nn, nn)
    N = nn ** 3
    h = 1.0 / nn
    L = 1.0
    k = _robin_k(D, L)
    x = disc.cell_centres(n)
    eta = np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]) * np.cos(k * (x[:, 2] - L / 2))
    lam = D * (2 * np.pi ** 2 + k ** 2) + mu
    A = disc.assemble(n, (0, 0, 0, 0, 1, 1), np.full(N, D), np.full(N, mu))
    eta_h = solvers.splu_solve(A, h ** 3 * lam * eta)
    return np.max(np.abs(eta_h - eta)) / np.max(np.abs(eta))


def _manufactured_error_2d(nn, D, mu):
    n = (nn, nn)
    N = nn * nn
    h = 1.0 / nn
    k = _robin_k(D, 1.0)
    x = disc.cell_centres(n)
    eta = np.cos(k * (x[:, 0] - 0.5)) * np.cos(k * (x[:, 1] - 0.5))
    lam = 2 * D * k ** 2 + mu
    A = disc.assemble(n, (1, 1, 1, 1), np.full(N, D), np.full(N, mu))
    eta_h = solvers.splu_solve(A, h ** 2 * lam * eta)
    return np.max(np.abs(eta_h - eta)) / np.max(np.abs(eta))


def test_robin_manufactured_solution_second_order_3d():
    e1 = _manufactured_error_3d(12, 0.3, 0.02)
    e2 = _manufactured_error_3d(24, 0.3, 0.02)
    assert e2 < 1e-2
    assert e1 / e2 > 3.3


def test_robin_manufactured_solution_second_order_2d():
    e1 = _manufactured_error_2d(16, 0.05, 0.01)
    e2 = _manufactured_error_2d(32, 0.05, 0.01)
    e3 = _manufactured_error_2d(64, 0.05, 0.01)
    assert e3 < 1e-3
    assert e1 / e2 > 3.3 and e2 / e3 > 3.3


def test_cell_numbering_and_centres():
    n = (4, 3, 2)
    x = disc.cell_centres(n)
    h = 0.25
    c = 1 + 4 * (2 + 3 * 1)     # i=1, j=2, k=1
    assert np.allclose(x[c], [(1.5) * h, 2.5 * h, 1.5 * h])


def test_diffusion_from_mua():
    assert disc.diffusion_from_mua(np.array([0.0]), 1.0)[0] == pytest.approx(1.0 / 3.0)
    assert disc.diffusion_from_mua(np.array([0.5]), 1.0)[0] == pytest.approx(1.0 / 4.5)


def test_layered_medium_flux_continuity():
    """D jumps from D1 to D2 across the cell faces at z = 1/4.  The exact solution
    sin(pi x) sin(pi y) f(z), with f = sin(k1 z) below and B sin(k2 (1 - z)) above,
    is continuous with continuous flux D f' (k2 solves D1 k1 cot(k1 z0) =
    -D2 k2 cot(k2 (1 - z0))).  The harmonic face mean keeps O(h^2); an
    arithmetic mean would fall to O(h) with a ~30x larger error."""
    D1, D2, mu, z0 = 0.05, 0.5, 0.02, 0.25
    k1 = np.pi
    k2 = sopt.brentq(lambda k: D1 * k1 / np.tan(k1 * z0) + D2 * k / np.tan(k * (1 - z0)),
                     1.0, np.pi / (1 - z0) - 1e-9)
    B = np.sin(k1 * z0) / np.sin(k2 * (1 - z0))

    def err(nn):
        n = (nn, nn, nn)
        x = disc.cell_centres(n)
        h = 1.0 / nn
        low = x[:, 2] < z0
        D = np.where(low, D1, D2)
        f = np.where(low, np.sin(k1 * x[:, 2]), B * np.sin(k2 * (1 - x[:, 2])))
        lam = np.where(low, D1 * (2 * np.pi ** 2 + k1 ** 2), D2 * (2 * np.pi ** 2 + k2 ** 2))
        eta = np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]) * f
        A = disc.assemble(n, (0,) * 6, D, np.full(nn ** 3, mu))
        eta_h = solvers.splu_solve(A, h ** 3 * (lam + mu) * eta)
        return np.max(np.abs(eta_h - eta)) / np.max(np.abs(eta))

    e16, e32 = err(16), err(32)
    assert e32 < 3e-3
    assert e16 / e32 > 3.2
