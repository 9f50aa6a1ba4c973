"""Workload descriptions: grid, boundary faces, PaLS lattice, optodes, sample sizes.

The five named workloads follow the problem sizes of the diffuse optical
tomography (DOT) model of Section 2 (box domain, Dirichlet lateral faces,
Robin top/bottom faces, zero frequency) and the experiments of Section 4
(RBF lattices with mixed-sign expansion coefficients, Fig. 3; 0.1% data noise).
The small ``t*`` workloads are parity-test sizes chosen to span several kernel
tiles with ragged tails.
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace

DIRICHLET = 0
ROBIN = 1

# parameter-activity bits per RBF: which of (alpha, beta, chi) are unknowns
ACT_ALPHA = 1
ACT_BETA = 2
ACT_CHI = 4


@dataclass(frozen=True)
class WorkloadConfig:
    name: str
    config_id: int
    dim: int                      # 2 or 3
    n: tuple                      # cells per axis (nx, ny[, nz])
    bc: tuple                     # per face -x,+x,-y,+y,-z,+z : DIRICHLET / ROBIN
    # absorption model constants (Section 2; readings for the unstated ones)
    mu_out: float = 0.01
    mu_in: float = 0.05
    mus_prime: float = 1.0
    cutoff: float = 0.15
    eps: float = 0.1
    gamma: float = 1e-3
    # RBF lattice
    lattice: tuple = (3, 3, 3)
    width: float = 0.3            # support radius 1/beta
    width_jitter: float = 0.0     # relative jitter of the width
    centre_jitter: float = 0.03
    centre_box: tuple = (0.0, 1.0)   # lattice spans this interval per axis
    alpha_mode: str = "mixed"     # "mixed": first half positive, rest negative; "positive"
    random_centres: bool = False  # C1: centres uniform in centre_box instead of a lattice
    active: int = ACT_ALPHA | ACT_BETA | ACT_CHI
    # optodes
    optodes: str = "faces"        # "faces": sources on z=0, detectors on z=max; "perimeter": co-located 2D
    src_lattice: tuple = (8, 8)
    det_lattice: tuple = (8, 8)
    n_perimeter: int = 16
    # simultaneous sources/detectors
    l_s: int = 8
    l_d: int = 8
    q_s: int = 0                  # optimized sources (0: purely random W)
    q_d: int = 0
    noise: float = 1e-3           # relative data noise (0.1%)
    # solver
    rtol: float = 1e-10
    theta_true_alpha_scale: float = 0.25
    theta_true_shift: float = 0.02
    theta_true_flip: int = 0      # RBFs whose expansion coefficient changes sign in the truth

    @property
    def N(self) -> int:
        out = 1
        for v in self.n:
            out *= v
        return out

    @property
    def m0(self) -> int:
        if self.random_centres:
            return self.n_rbf
        out = 1
        for v in self.lattice[: self.dim]:
            out *= v
        return out

    n_rbf: int = 4

    @property
    def n_active_per_rbf(self) -> int:
        k = 0
        if self.active & ACT_ALPHA:
            k += 1
        if self.active & ACT_BETA:
            k += 1
        if self.active & ACT_CHI:
            k += self.dim
        return k

    @property
    def n_p(self) -> int:
        return self.m0 * self.n_active_per_rbf

    @property
    def n_s(self) -> int:
        if self.optodes == "perimeter":
            return self.n_perimeter
        return self.src_lattice[0] * self.src_lattice[1]

    @property
    def n_d(self) -> int:
        if self.optodes == "perimeter":
            return self.n_perimeter
        return self.det_lattice[0] * self.det_lattice[1]


_ROBIN_Z = (DIRICHLET, DIRICHLET, DIRICHLET, DIRICHLET, ROBIN, ROBIN)

CONFIGS = {
    # 2D, 32x32, Robin on all faces, 4 RBFs (alpha + centre active: 12 params),
    # 16 co-located perimeter optodes, full (unsampled) W = V = I.
    "C1": WorkloadConfig(
        name="C1", config_id=1, dim=2, n=(32, 32), bc=(ROBIN, ROBIN, ROBIN, ROBIN, ROBIN, ROBIN),
        random_centres=True, n_rbf=4, centre_box=(0.2, 0.8), width=0.1, width_jitter=0.2,
        alpha_mode="positive", active=ACT_ALPHA | ACT_CHI, optodes="perimeter", n_perimeter=16,
        l_s=16, l_d=16, rtol=1e-12,
    ),
    # 3D 64^3, 27 RBFs (alpha + centre: 108 params), 8x8 sources / 8x8 detectors, l = 8.
    "C2": WorkloadConfig(
        name="C2", config_id=2, dim=3, n=(64, 64, 64), bc=_ROBIN_Z, lattice=(3, 3, 3), width=0.3,
        centre_jitter=0.03, active=ACT_ALPHA | ACT_CHI, src_lattice=(8, 8), det_lattice=(8, 8),
        l_s=8, l_d=8, rtol=1e-10,
    ),
    # 3D 128^3, 64 RBFs (320 params), 16x16 / 16x16 optodes, l = 20 = 10 optimized + 10 random.
    "C3": WorkloadConfig(
        name="C3", config_id=3, dim=3, n=(128, 128, 128), bc=_ROBIN_Z, lattice=(4, 4, 4), width=0.25,
        centre_jitter=0.03, src_lattice=(16, 16), det_lattice=(16, 16), l_s=20, l_d=20, q_s=10,
        q_d=10, rtol=1e-8,
    ),
    # 3D 96^3, 100 RBFs (500 params), 16x8 / 16x8 optodes, l = 16.
    "C4": WorkloadConfig(
        name="C4", config_id=4, dim=3, n=(96, 96, 96), bc=_ROBIN_Z, lattice=(5, 5, 4), width=0.2,
        centre_jitter=0.03, src_lattice=(16, 8), det_lattice=(16, 8), l_s=16, l_d=16, rtol=1e-10,
    ),
    # 3D 128^3, 1000 RBFs (5000 params), 16x16 / 16x16 optodes, l = 40 (1600 sampled rows).
    "C5": WorkloadConfig(
        name="C5", config_id=5, dim=3, n=(128, 128, 128), bc=_ROBIN_Z, lattice=(10, 10, 10),
        width=0.1, centre_jitter=0.02, src_lattice=(16, 16), det_lattice=(16, 16), l_s=40, l_d=40,
        rtol=1e-8,
    ),
}

# Parity-test workloads: small enough for the oracle's direct solver, ragged
# against every tile size used by the kernels (tiles are powers of two).
TEST_CONFIGS = {
    "t2d": WorkloadConfig(
        name="t2d", config_id=101, dim=2, n=(37, 29), bc=(ROBIN, ROBIN, DIRICHLET, ROBIN, ROBIN, ROBIN),
        random_centres=True, n_rbf=5, centre_box=(0.2, 0.8), width=0.2, width_jitter=0.2,
        alpha_mode="mixed", active=ACT_ALPHA | ACT_BETA | ACT_CHI, optodes="perimeter",
        n_perimeter=12, l_s=5, l_d=4, rtol=1e-12,
    ),
    "t3d": WorkloadConfig(
        name="t3d", config_id=102, dim=3, n=(19, 13, 11), bc=_ROBIN_Z, lattice=(2, 2, 2), width=0.45,
        centre_jitter=0.03, src_lattice=(4, 3), det_lattice=(3, 4), l_s=4, l_d=3, rtol=1e-12,
    ),
    "t3d_b": WorkloadConfig(
        name="t3d_b", config_id=103, dim=3, n=(24, 24, 24), bc=(ROBIN, DIRICHLET, DIRICHLET, ROBIN, ROBIN, ROBIN),
        lattice=(3, 3, 3), width=0.3, centre_jitter=0.03, src_lattice=(5, 5), det_lattice=(4, 4),
        l_s=6, l_d=5, q_s=2, q_d=2, rtol=1e-12,
    ),
    "t3d_c": WorkloadConfig(
        name="t3d_c", config_id=104, dim=3, n=(70, 33, 17), bc=_ROBIN_Z, lattice=(4, 3, 2), width=0.3,
        centre_jitter=0.03, src_lattice=(6, 4), det_lattice=(5, 5), l_s=9, l_d=7, rtol=1e-12,
    ),
}


# Inversion workloads (the outer Gauss-Newton driver of Sections 3.2 and 4).
# The unit box stands for a 60 mm slab: with x = L x', L = 60 mm, the diffusion
# equation and its Robin condition keep their form on [0, 1]^3 with D' = D / L
# and mu' = L mu, which is D = 1 / (3 (mu + mus')) with mu and mus' both scaled
# by L.  Background absorption 0.01 / mm, anomaly 0.05 / mm and reduced
# scattering 1 / mm (breast-tissue values) then give a diffusion length of
# about 6 mm, so absorption anomalies are visible in the data; the initial
# guess is the reference lattice (Fig. 3 layout: mixed-sign expansion
# coefficients) and the truth rescales, moves and flips some of its RBFs.
_L_MM = 60.0
INVERSION_CONFIGS = {
    # parity-test size for the driver (the oracle replays it with direct solves)
    "inv_t": WorkloadConfig(
        name="inv_t", config_id=201, dim=3, n=(24, 24, 24), bc=_ROBIN_Z, lattice=(3, 3, 3),
        width=0.3, centre_jitter=0.03, src_lattice=(6, 6), det_lattice=(6, 6), l_s=6, l_d=6,
        q_s=2, q_d=2, mu_out=0.01 * _L_MM, mu_in=0.05 * _L_MM, mus_prime=1.0 * _L_MM,
        theta_true_alpha_scale=0.5, theta_true_shift=0.05, theta_true_flip=3, rtol=1e-12,
    ),
    # Example 2's shape (table T3): 32^3, 225 sources on top, 225 detectors on
    # the bottom, 27 RBFs with five parameters each (135), 12 simultaneous
    # sources and detectors, 2 of them optimized after the SAA phase
    "inv_x2": WorkloadConfig(
        name="inv_x2", config_id=202, dim=3, n=(32, 32, 32), bc=_ROBIN_Z, lattice=(3, 3, 3),
        width=0.3, centre_jitter=0.03, src_lattice=(15, 15), det_lattice=(15, 15), l_s=12,
        l_d=12, q_s=2, q_d=2, mu_out=0.01 * _L_MM, mu_in=0.05 * _L_MM, mus_prime=1.0 * _L_MM,
        theta_true_alpha_scale=0.5, theta_true_shift=0.05, theta_true_flip=3, rtol=1e-10,
    ),
}


def get_config(name: str, **overrides) -> WorkloadConfig:
    if name in CONFIGS:
        cfg = CONFIGS[name]
    elif name in TEST_CONFIGS:
        cfg = TEST_CONFIGS[name]
    elif name in INVERSION_CONFIGS:
        cfg = INVERSION_CONFIGS[name]
    else:
        raise KeyError(f"unknown workload {name!r}")
    return replace(cfg, **overrides) if overrides else cfg
