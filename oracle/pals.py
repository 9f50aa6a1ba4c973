"""Parametric level set (PaLS) absorption and its parameter derivatives.

Section 2: phi(x; p) = sum_j alpha_j psi(|| beta_j (x - chi_j) ||_dagger) with
the regularized norm ||y||_dagger = sqrt(||y||^2 + gamma^2) and the Wendland
function psi_{2,1}(r) = (1 - r)^4 (4 r + 1) for r < 1, 0 otherwise (footnote
to the PaLS definition).  The absorption (eq. absorption const) is
mu = mu_in H_eps(phi - c) + mu_out (1 - H_eps(phi - c)).

Readings (the paper does not define H_eps, eps or gamma):
  H_eps(s) = 0 for s < -eps, 1 for s > eps, and
             (1 + s/eps + sin(pi s / eps) / pi) / 2 in between (C^1);
  delta_eps(s) = H_eps'(s) = (1 + cos(pi s / eps)) / (2 eps) on |s| <= eps.
Parameters are stored RBF-major, theta[j] = [alpha_j, beta_j, chi_j (d)].
The unknowns of the inversion are a subset selected per RBF by an activity
mask (bit 0 alpha, bit 1 beta, bit 2 chi); parameter k = j * n_act + local
index in the order alpha, beta, chi_1..chi_d.
"""

from __future__ import annotations

import numpy as np

ACT_ALPHA, ACT_BETA, ACT_CHI = 1, 2, 4


def wendland(r):
    """psi_{2,1}(r) = (1 - r)^4 (4 r + 1) on [0, 1), zero beyond."""
    r = np.asarray(r, dtype=np.float64)
    return np.where(r < 1.0, (1.0 - r) ** 4 * (4.0 * r + 1.0), 0.0)


def wendland_prime(r):
    """psi'(r) = -20 r (1 - r)^3 on [0, 1), zero beyond."""
    r = np.asarray(r, dtype=np.float64)
    return np.where(r < 1.0, -20.0 * r * (1.0 - r) ** 3, 0.0)


def heaviside_eps(s, eps: float):
    s = np.asarray(s, dtype=np.float64)
    mid = 0.5 * (1.0 + s / eps + np.sin(np.pi * s / eps) / np.pi)
    return np.where(s < -eps, 0.0, np.where(s > eps, 1.0, mid))


def delta_eps(s, eps: float):
    s = np.asarray(s, dtype=np.float64)
    return np.where(np.abs(s) <= eps, (1.0 + np.cos(np.pi * s / eps)) / (2.0 * eps), 0.0)


def rbf_radius(x: np.ndarray, theta_j: np.ndarray, gamma: float) -> np.ndarray:
    """r_j(x) = sqrt(beta_j^2 ||x - chi_j||^2 + gamma^2) for every row of x."""
    beta, chi = theta_j[1], theta_j[2:]
    rho2 = np.sum((x - chi) ** 2, axis=1)
    return np.sqrt(beta * beta * rho2 + gamma * gamma)


def phi(x: np.ndarray, theta: np.ndarray, gamma: float) -> np.ndarray:
    """Level-set function at the points x (N, d)."""
    out = np.zeros(x.shape[0])
    for j in range(theta.shape[0]):
        out += theta[j, 0] * wendland(rbf_radius(x, theta[j], gamma))
    return out


def mua(x: np.ndarray, theta: np.ndarray, mu_in: float, mu_out: float, cutoff: float,
        eps: float, gamma: float) -> np.ndarray:
    """mu(x; p) of eq. (absorption const)."""
    H = heaviside_eps(phi(x, theta, gamma) - cutoff, eps)
    return mu_in * H + mu_out * (1.0 - H)


def n_active(active: int, d: int) -> int:
    return (1 if active & ACT_ALPHA else 0) + (1 if active & ACT_BETA else 0) + \
        (d if active & ACT_CHI else 0)


def dphi_dtheta_j(x: np.ndarray, theta_j: np.ndarray, gamma: float) -> np.ndarray:
    """All 2 + d partial derivatives of alpha_j psi(r_j(x)), shape (N, 2 + d).

    d/d alpha  = psi(r)
    d/d beta   = alpha psi'(r) beta rho^2 / r   = -20 alpha beta rho^2 (1 - r)^3
    d/d chi_m  = alpha psi'(r) beta^2 (chi_m - x_m) / r
               = 20 alpha beta^2 (x_m - chi_m) (1 - r)^3
    (zero where r >= 1).
    """
    alpha, beta, chi = theta_j[0], theta_j[1], theta_j[2:]
    diff = x - chi
    rho2 = np.sum(diff ** 2, axis=1)
    r = np.sqrt(beta * beta * rho2 + gamma * gamma)
    inside = r < 1.0
    omr3 = np.where(inside, (1.0 - r) ** 3, 0.0)
    out = np.empty((x.shape[0], theta_j.size))
    out[:, 0] = wendland(r)
    out[:, 1] = -20.0 * alpha * beta * rho2 * omr3
    out[:, 2:] = 20.0 * alpha * beta * beta * diff * omr3[:, None]
    return out


def active_columns(active: int, d: int) -> list:
    """Indices into [alpha, beta, chi_1..chi_d] that are unknowns, in order."""
    cols = []
    if active & ACT_ALPHA:
        cols.append(0)
    if active & ACT_BETA:
        cols.append(1)
    if active & ACT_CHI:
        cols += list(range(2, 2 + d))
    return cols


def dmua_dp(x: np.ndarray, theta: np.ndarray, active: int, mu_in: float, mu_out: float,
            cutoff: float, eps: float, gamma: float) -> np.ndarray:
    """Dense (N, n_p) matrix of d mu / d p_k at the points x.

    d mu / d p_k = (mu_in - mu_out) delta_eps(phi - c) d phi / d p_k.
    """
    d = x.shape[1]
    cols = active_columns(active, d)
    na = len(cols)
    band = (mu_in - mu_out) * delta_eps(phi(x, theta, gamma) - cutoff, eps)
    out = np.zeros((x.shape[0], theta.shape[0] * na))
    for j in range(theta.shape[0]):
        dj = dphi_dtheta_j(x, theta[j], gamma)
        out[:, j * na:(j + 1) * na] = band[:, None] * dj[:, cols]
    return out


def theta_from_params(theta: np.ndarray, params: np.ndarray, active: int) -> np.ndarray:
    """Scatter an n_p vector of unknowns back into a full theta array."""
    d = theta.shape[1] - 2
    cols = active_columns(active, d)
    out = theta.copy()
    out[:, cols] = np.asarray(params).reshape(theta.shape[0], len(cols))
    return out


def params_from_theta(theta: np.ndarray, active: int) -> np.ndarray:
    d = theta.shape[1] - 2
    return theta[:, active_columns(active, d)].reshape(-1).copy()
