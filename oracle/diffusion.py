"""Inverting for diffusion as well (Section 3.3, last paragraph: dA/dp_k has
5 (2D) or 7 (3D) diagonals when the diffusion coefficient is an unknown too).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading: the level set describes an anomaly in both optical properties, the
absorption mu and the reduced scattering mu_s' (PaLS with the same smoothed
Heaviside, eq. absorption const applied to each):
    mu   = mu_out  + (mu_in  - mu_out ) H_eps(phi - c)
    mu_s = mus_out + (mus_in - mus_out) H_eps(phi - c)
    D    = 1 / (3 (mu + mu_s))            (diffusion approximation)
so D is no longer frozen and A(p) = -div(D(p) grad) + mu(p).  Then
    d mu / d p_k = (mu_in - mu_out) delta_eps(phi - c) d phi / d p_k,
    d D  / d p_k = -3 D^2 ((mu_in - mu_out) + (mus_in - mus_out))
                     delta_eps(phi - c) d phi / d p_k,
and dA/dp_k follows from the finite-volume coefficients by the chain rule:
    interior face c|c': d T / d D_c = h^(d-2) 2 D_c'^2 / (D_c + D_c')^2
    Dirichlet face:     d T / d D_c = h^(d-2) 2
    Robin face:         d T / d D_c = h^(d-1) 2 h / (h + 4 D_c)^2
    dA/dp_k = sum_faces dT_f/dp_k (e_c - e_c')(e_c - e_c')^T
              + sum_boundary dT_b/dp_k e_c e_c^T + h^d diag(d mu / d p_k).
The sampled Jacobian keeps eq. Jacobian kth column with this matrix:
J_s[j + l_d i, k] = - z_j^T (dA/dp_k) u_i.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import discretization as disc
from . import pals


def coefficients(prob, theta, mus_in: float, mus_out: float):
    """mu, D and the level-set factors at the cell centres."""
    c = prob.consts
    ph = pals.phi(prob.x, theta, c["gamma"])
    H = pals.heaviside_eps(ph - c["cutoff"], c["eps"])
    mu = c["mu_in"] * H + c["mu_out"] * (1.0 - H)
    mus = mus_in * H + mus_out * (1.0 - H)
    return mu, 1.0 / (3.0 * (mu + mus)), ph


def operator(prob, theta, mus_in: float, mus_out: float) -> sp.csr_matrix:
    mu, D, _ = coefficients(prob, theta, mus_in, mus_out)
    return disc.assemble(prob.n, prob.bc, D, mu)


def derivative_fields(prob, theta, mus_in: float, mus_out: float):
    """(N, n_p) matrices d mu / d p and d D / d p."""
    c = prob.consts
    mu, D, _ = coefficients(prob, theta, mus_in, mus_out)
    dmu = pals.dmua_dp(prob.x, theta, prob.active, **c)
    ratio = 1.0 + (mus_in - mus_out) / (c["mu_in"] - c["mu_out"])
    dD = -3.0 * (D * D * ratio)[:, None] * dmu
    return D, dmu, dD


def dA_dp(prob, D: np.ndarray, dD: np.ndarray, dmu: np.ndarray) -> sp.csr_matrix:
    """The derivative of the assembled A along one parameter (dD, dmu: (N,))."""
    n, bc, d = prob.n, prob.bc, len(prob.n)
    h = disc.spacing(n)
    N = int(np.prod(n))
    shape = disc.cell_shape(n)
    Dg, dDg = D.reshape(shape), dD.reshape(shape)
    idx = np.arange(N).reshape(shape)
    diag = h ** d * np.asarray(dmu, dtype=np.float64).copy()
    rows, cols, vals = [], [], []
    for a in range(d):
        ax = d - 1 - a
        lo = [slice(None)] * d
        hi = [slice(None)] * d
        lo[ax] = slice(0, n[a] - 1)
        hi[ax] = slice(1, n[a])
        Dl, Dh = Dg[tuple(lo)], Dg[tuple(hi)]
        dl, dh = dDg[tuple(lo)], dDg[tuple(hi)]
        dT = (h ** (d - 2) * 2.0 * (Dh * Dh * dl + Dl * Dl * dh) / (Dl + Dh) ** 2).ravel()
        c0, c1 = idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel()
        np.add.at(diag, c0, dT)
        np.add.at(diag, c1, dT)
        rows += [c0, c1]
        cols += [c1, c0]
        vals += [-dT, -dT]
        for side, sl in ((2 * a, slice(0, 1)), (2 * a + 1, slice(n[a] - 1, n[a]))):
            s = [slice(None)] * d
            s[ax] = sl
            Db, dDb = Dg[tuple(s)].ravel(), dDg[tuple(s)].ravel()
            cb = idx[tuple(s)].ravel()
            if bc[side] == 0:
                dTb = h ** (d - 2) * 2.0 * dDb
            else:
                dTb = h ** (d - 1) * 2.0 * h * dDb / (h + 4.0 * Db) ** 2
            np.add.at(diag, cb, dTb)
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    M.sum_duplicates()
    return M


def jacobian(prob, theta, mus_in: float, mus_out: float, U: np.ndarray, Z: np.ndarray):
    """J_s[j + l_d i, k] = - z_j^T (dA/dp_k) u_i, loop over parameters."""
    D, dmu, dD = derivative_fields(prob, theta, mus_in, mus_out)
    ls, ld = U.shape[1], Z.shape[1]
    J = np.zeros((ls * ld, dmu.shape[1]))
    for k in range(dmu.shape[1]):
        if not np.any(dmu[:, k]):
            continue
        Mk = dA_dp(prob, D, dD[:, k], dmu[:, k])
        B = -(np.asarray(Z).T @ (Mk @ np.asarray(U)))      # (ld, ls): [j, i]
        J[:, k] = B.reshape(-1, order="F")
    return J
