"""Pins for the oracle's PaLS absorption model (Section 2).

* Wendland psi_{2,1} and psi' at exact dyadic points (golden fixture);
* smoothed Heaviside: end values, midpoint, C^1 continuity, delta integrates to 1;
* level set at an RBF centre equals alpha psi(gamma) in closed form;
* d mu / d p against central finite differences of mu itself, for every
  parameter kind (alpha, beta, chi) in 2D and 3D.
"""

import os

import numpy as np
import pytest
import scipy.integrate as sint

from oracle import pals

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "wendland_psi21.txt")


def test_wendland_golden_values():
    tab = np.loadtxt(GOLDEN)
    r, psi, dpsi = tab[:, 0], tab[:, 1], tab[:, 2]
    assert np.array_equal(pals.wendland(r), psi)
    assert np.array_equal(pals.wendland_prime(r), dpsi)


def test_wendland_derivative_matches_fd():
    r = np.linspace(0.01, 0.99, 37)
    h = 1e-6
    fd = (pals.wendland(r + h) - pals.wendland(r - h)) / (2 * h)
    assert np.allclose(fd, pals.wendland_prime(r), rtol=0, atol=1e-8)


def test_heaviside_and_delta():
    eps = 0.1
    assert pals.heaviside_eps(0.0, eps) == pytest.approx(0.5)
    assert pals.heaviside_eps(-eps, eps) == pytest.approx(0.0, abs=1e-15)
    assert pals.heaviside_eps(eps, eps) == pytest.approx(1.0)
    assert pals.heaviside_eps(-0.3, eps) == 0.0 and pals.heaviside_eps(0.3, eps) == 1.0
    assert pals.delta_eps(0.0, eps) == pytest.approx(1.0 / eps)
    assert pals.delta_eps(eps, eps) == pytest.approx(0.0, abs=1e-12)
    val, _ = sint.quad(lambda s: float(pals.delta_eps(s, eps)), -eps, eps)
    assert val == pytest.approx(1.0, abs=1e-12)
    s = np.linspace(-0.2, 0.2, 81)
    h = 1e-7
    fd = (pals.heaviside_eps(s + h, eps) - pals.heaviside_eps(s - h, eps)) / (2 * h)
    assert np.allclose(fd, pals.delta_eps(s, eps), atol=1e-6)


def test_phi_at_centre_closed_form():
    gamma = 1e-3
    theta = np.array([[1.3, 4.0, 0.5, 0.25, 0.75]])
    x = theta[:, 2:].copy()
    r = gamma
    expect = 1.3 * (1 - r) ** 4 * (4 * r + 1)
    assert pals.phi(x, theta, gamma)[0] == pytest.approx(expect, rel=1e-15)
    far = np.array([[0.5, 0.25, 0.75 + 0.26]])   # beta * dist = 1.04 > 1
    assert pals.phi(far, theta, gamma)[0] == 0.0


def test_mua_limits():
    theta = np.array([[1.5, 5.0, 0.5, 0.5]])
    x = np.array([[0.5, 0.5], [0.95, 0.95]])
    mu = pals.mua(x, theta, mu_in=0.05, mu_out=0.01, cutoff=0.15, eps=0.1, gamma=1e-3)
    assert mu[0] == pytest.approx(0.05) and mu[1] == pytest.approx(0.01)


@pytest.mark.parametrize("d,active", [(2, 7), (3, 7), (3, 5), (2, 5)])
def test_dmua_dp_matches_central_fd(d, active):
    rng = np.random.default_rng(11 + d)
    m0 = 3
    theta = np.empty((m0, 2 + d))
    theta[:, 0] = [0.9, -0.7, 1.2]
    theta[:, 1] = rng.uniform(2.5, 4.0, m0)
    theta[:, 2:] = rng.uniform(0.3, 0.7, (m0, d))
    x = rng.uniform(0.0, 1.0, (400, d))
    consts = dict(mu_in=0.05, mu_out=0.01, cutoff=0.15, eps=0.1, gamma=1e-3)
    G = pals.dmua_dp(x, theta, active, **consts)
    p0 = pals.params_from_theta(theta, active)
    assert G.shape == (400, p0.size)
    hstep = 1e-6
    for k in range(p0.size):
        pp, pm = p0.copy(), p0.copy()
        pp[k] += hstep
        pm[k] -= hstep
        mp = pals.mua(x, pals.theta_from_params(theta, pp, active), **consts)
        mm = pals.mua(x, pals.theta_from_params(theta, pm, active), **consts)
        fd = (mp - mm) / (2 * hstep)
        scale = max(np.abs(G[:, k]).max(), 1e-3)
        assert np.max(np.abs(fd - G[:, k])) <= 2e-6 * scale, k
    # a band cell exists for every RBF, so every column is exercised
    assert np.all(np.abs(G).max(axis=0) > 0)
