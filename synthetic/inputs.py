"""Seeded random draws and optode geometry for a workload.

Seeds: ``numpy.random.SeedSequence(170605586 + config_id)`` spawns one child
stream per quantity, in this order: reference parameters, true parameters,
source signs W, detector signs V, data noise, complementary source signs,
complementary detector signs.  Changing one quantity's recipe never changes
another's draws.

Everything returned is raw: Rademacher signs are +-1 integers (the 1/sqrt(l)
scaling of the simultaneous-source matrices is applied by the consumers),
the noise is standard normal, and the parameters are stored RBF-major as
``[alpha, beta, chi_1 .. chi_d]`` per basis function.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .configs import WorkloadConfig

BASE_SEED = 170605586


@dataclass
class Workload:
    cfg: WorkloadConfig
    theta_ref: np.ndarray     # (m0, 2 + d) float64: [alpha, beta, chi...]
    theta_true: np.ndarray    # (m0, 2 + d) float64
    src_cells: np.ndarray     # (n_s,) int32 linear cell index i + nx*(j + ny*k)
    det_cells: np.ndarray     # (n_d,) int32
    w_signs: np.ndarray       # (n_s, l_s) int8 in {-1, +1}
    v_signs: np.ndarray       # (n_d, l_d) int8
    y_signs: np.ndarray       # (n_s - q_s, l_s - q_s) int8 (complementary sources)
    z_signs: np.ndarray       # (n_d - q_d, l_d - q_d) int8 (complementary detectors)
    xi: np.ndarray            # (n_d, n_s) float64 standard normal data noise


def _rademacher(rng: np.random.Generator, shape) -> np.ndarray:
    return (rng.integers(0, 2, size=shape, dtype=np.int8) * 2 - 1).astype(np.int8)


def _lattice_centres(cfg: WorkloadConfig, rng: np.random.Generator) -> np.ndarray:
    d = cfg.dim
    lo, hi = cfg.centre_box
    if cfg.random_centres:
        return rng.uniform(lo, hi, size=(cfg.m0, d))
    axes = [lo + (hi - lo) * (np.arange(cfg.lattice[a]) + 0.5) / cfg.lattice[a] for a in range(d)]
    grids = np.meshgrid(*axes, indexing="ij")
    # first axis fastest in the RBF numbering
    pts = np.stack([g.transpose(tuple(range(d))[::-1]).reshape(-1) for g in grids], axis=1)
    pts = pts + rng.uniform(-cfg.centre_jitter, cfg.centre_jitter, size=pts.shape)
    return pts


def _theta_ref(cfg: WorkloadConfig, rng: np.random.Generator) -> np.ndarray:
    m0, d = cfg.m0, cfg.dim
    centres = _lattice_centres(cfg, rng)
    mag = rng.uniform(0.5, 1.5, size=m0)
    if cfg.alpha_mode == "positive":
        sign = np.ones(m0)
    else:
        sign = -np.ones(m0)
        sign[rng.permutation(m0)[: m0 // 2]] = 1.0
    width = cfg.width * rng.uniform(1.0 - cfg.width_jitter, 1.0 + cfg.width_jitter, size=m0)
    theta = np.empty((m0, 2 + d))
    theta[:, 0] = sign * mag
    theta[:, 1] = 1.0 / width
    theta[:, 2:] = centres
    return theta


def _theta_true(cfg: WorkloadConfig, theta_ref: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    theta = theta_ref.copy()
    theta[:, 0] *= 1.0 + rng.uniform(-cfg.theta_true_alpha_scale, cfg.theta_true_alpha_scale, size=cfg.m0)
    theta[:, 2:] += rng.uniform(-cfg.theta_true_shift, cfg.theta_true_shift, size=theta[:, 2:].shape)
    if cfg.theta_true_flip > 0:
        # basis functions that change sides (visible <-> invisible) in the truth
        theta[rng.permutation(cfg.m0)[: cfg.theta_true_flip], 0] *= -1.0
    return theta


def _cell_index(cfg: WorkloadConfig, ijk) -> int:
    n = cfg.n
    if cfg.dim == 2:
        i, j = ijk
        return int(i + n[0] * j)
    i, j, k = ijk
    return int(i + n[0] * (j + n[1] * k))


def _face_lattice(cfg: WorkloadConfig, lat, z_layer: int) -> np.ndarray:
    nx, ny = cfg.n[0], cfg.n[1]
    cells = []
    for b in range(lat[1]):
        for a in range(lat[0]):
            i = int(np.floor((a + 0.5) * nx / lat[0]))
            j = int(np.floor((b + 0.5) * ny / lat[1]))
            cells.append(_cell_index(cfg, (i, j, z_layer)))
    return np.asarray(cells, dtype=np.int32)


def _perimeter(cfg: WorkloadConfig) -> np.ndarray:
    """Co-located optodes evenly spaced along the boundary of the unit square."""
    nx, ny = cfg.n[0], cfg.n[1]
    P = cfg.n_perimeter
    cells = []
    for k in range(P):
        s = (k + 0.5) * 4.0 / P
        edge, t = int(np.floor(s)), s - np.floor(s)
        if edge == 0:      # bottom, left to right
            i, j = int(t * nx), 0
        elif edge == 1:    # right, bottom to top
            i, j = nx - 1, int(t * ny)
        elif edge == 2:    # top, right to left
            i, j = int((1.0 - t) * nx), ny - 1
        else:              # left, top to bottom
            i, j = 0, int((1.0 - t) * ny)
        i, j = min(i, nx - 1), min(j, ny - 1)
        cells.append(_cell_index(cfg, (i, j)))
    return np.asarray(cells, dtype=np.int32)


def make_workload(cfg: WorkloadConfig) -> Workload:
    ss = np.random.SeedSequence(BASE_SEED + cfg.config_id)
    kids = ss.spawn(7)
    rng = [np.random.default_rng(k) for k in kids]
    theta_ref = _theta_ref(cfg, rng[0])
    theta_true = _theta_true(cfg, theta_ref, rng[1])
    if cfg.optodes == "perimeter":
        src = _perimeter(cfg)
        det = src.copy()
    else:
        src = _face_lattice(cfg, cfg.src_lattice, 0)
        det = _face_lattice(cfg, cfg.det_lattice, cfg.n[2] - 1)
    n_s, n_d = src.size, det.size
    w = _rademacher(rng[2], (n_s, cfg.l_s))
    v = _rademacher(rng[3], (n_d, cfg.l_d))
    xi = rng[4].standard_normal((n_d, n_s))
    y = _rademacher(rng[5], (n_s - cfg.q_s, cfg.l_s - cfg.q_s))
    z = _rademacher(rng[6], (n_d - cfg.q_d, cfg.l_d - cfg.q_d))
    return Workload(cfg=cfg, theta_ref=theta_ref, theta_true=theta_true, src_cells=src,
                    det_cells=det, w_signs=w, v_signs=v, y_signs=y, z_signs=z, xi=xi)


def sketch_draws(n_s: int, n_d: int, n_p: int, q_s: int, q_d: int, k: int, sweeps: int,
                 seed: int) -> dict:
    """Random test vectors of the sketched optimized design: Rademacher source
    signs w1 (n_s x k), and standard normal parameter directions t1, t2[s],
    t3[s] (n_p x k) and coefficient vectors a2[s] (q_d x k), a3[s] (q_s x k)
    per sweep s.  Raw draws only."""
    rng = np.random.default_rng(np.random.SeedSequence(BASE_SEED + 7919 * seed))
    out = {"w1": _rademacher(rng, (n_s, k)).astype(np.float64),
           "t1": rng.standard_normal((n_p, k)), "a2": [], "t2": [], "a3": [], "t3": []}
    for _ in range(sweeps):
        out["a2"].append(rng.standard_normal((q_d, k)))
        out["t2"].append(rng.standard_normal((n_p, k)))
        out["a3"].append(rng.standard_normal((q_s, k)))
        out["t3"].append(rng.standard_normal((n_p, k)))
    return out

