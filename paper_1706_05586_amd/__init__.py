"""MI355X (gfx950) hot path of randomized DOT inversion with random and optimized
simultaneous sources and detectors: multi-RHS diffusion solves, PaLS absorption,
sampled misfit, Jacobian contraction and adjoint gradient, behind the C ABI
declared in include/dotpath.h.  The HIP library libdotpath.so is required.
"""

from ._lib import (DOT_ACT_ALPHA, DOT_ACT_BETA, DOT_ACT_CHI, DOT_BC_DIRICHLET, DOT_BC_ROBIN,
                   DOT_FP64, DOT_JAC_FP64, DOT_JAC_SPLIT_BF16, DOT_JAC_SPLIT_BF16X3, DOT_MIXED,
                   DOT_PRECOND_AUTO, DOT_PRECOND_JACOBI, DOT_PRECOND_MG, DOT_PRECOND_MG_F32,
                   DOT_PROF_JACOBIAN, DOT_PROF_PCG1_FP32, DOT_PROF_PCG1_FP64, DOT_PROF_PCG2_FP32,
                   DOT_PROF_PCG2_FP64, DOT_PROF_RESID, DOT_PROF_VCYCLE_FP32, DOT_PROF_VCYCLE_FP64,
                   DotError, NotConverged, LIB_PATH)
from .api import (Grid, Operator, Pals, SolveResult, colmajor, empty_colmajor, gemm, hooi,
                  mode_gram, optimized_design, pals_field, qr_complete, svd_thin, symeig,
                  tsvd_step)
from .autograd import MisfitFn, MisfitProblem, misfit
from . import inversion  # noqa: E402  (outer Gauss-Newton driver on the ABI calls)

__all__ = [
    "DOT_ACT_ALPHA", "DOT_ACT_BETA", "DOT_ACT_CHI", "DOT_BC_DIRICHLET", "DOT_BC_ROBIN",
    "DOT_FP64", "DOT_MIXED", "DOT_PRECOND_AUTO", "DOT_PRECOND_JACOBI", "DOT_PRECOND_MG", "DOT_PRECOND_MG_F32", "DOT_JAC_FP64", "DOT_JAC_SPLIT_BF16", "DOT_JAC_SPLIT_BF16X3", "DotError", "NotConverged",
    "DOT_PROF_JACOBIAN", "DOT_PROF_PCG1_FP32", "DOT_PROF_PCG1_FP64", "DOT_PROF_PCG2_FP32",
    "DOT_PROF_PCG2_FP64", "DOT_PROF_RESID", "DOT_PROF_VCYCLE_FP32", "DOT_PROF_VCYCLE_FP64",
    "LIB_PATH", "Grid", "Operator", "Pals", "SolveResult", "colmajor", "empty_colmajor",
    "gemm", "pals_field", "MisfitFn", "MisfitProblem", "misfit", "mode_gram", "symeig",
    "qr_complete", "hooi", "svd_thin", "tsvd_step", "optimized_design", "inversion",
]
