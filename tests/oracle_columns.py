"""Oracle columns of dA/dp on one RBF's support at full grid sizes (test support).

At 64^3 - 128^3 the oracle's dense N x n_p matrix of d mu / d p does not fit
comfortably, so the full-size tests evaluate it only on the bounding box of
one RBF's support, with the oracle's own PaLS functions, and compare the GPU
Jacobian and gradient columns of that RBF with the oracle's sparse loop nest
and adjoint form on the fields gathered there.
"""

import numpy as np

from oracle import discretization as odisc
from oracle import pals as opals


def support_columns(wl, m, theta=None):
    """Cells of RBF m's support box and the oracle's h^3 dmu/dp columns of
    its active parameters there (rows that are zero are dropped), at theta
    (default: the workload's reference parameters)."""
    cfg = wl.cfg
    th = wl.theta_ref if theta is None else np.asarray(theta)
    cols = opals.active_columns(cfg.active, cfg.dim)
    n = tuple(cfg.n)
    h = odisc.spacing(n)
    R = 1.0 / abs(th[m, 1])
    lo = np.maximum(0, np.floor((th[m, 2:] - R) / h - 0.5).astype(int))
    hi = np.minimum(np.array(n) - 1, np.ceil((th[m, 2:] + R) / h - 0.5).astype(int))
    axes = [np.arange(lo[a], hi[a] + 1) for a in range(3)]
    gz, gy, gx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    cells = (gx + n[0] * (gy + n[1] * gz)).ravel()
    x = np.stack([(gx.ravel() + 0.5) * h, (gy.ravel() + 0.5) * h, (gz.ravel() + 0.5) * h], 1)
    band = (cfg.mu_in - cfg.mu_out) * opals.delta_eps(
        opals.phi(x, th, cfg.gamma) - cfg.cutoff, cfg.eps)
    G = h ** 3 * band[:, None] * opals.dphi_dtheta_j(x, th[m], cfg.gamma)[:, cols]
    keep = np.any(G != 0, axis=1)
    return cells[keep], G[keep], len(cols)
