"""ctypes declarations for libdotpath.so (the C ABI in include/dotpath.h).

The shared library is required: importing this module raises ImportError when
it has not been built (``python -c "import __graft_entry__ as g; g.build()"``
or ``python paper_1706_05586_amd/build.py``).  There is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdotpath.so")

DOT_OK = 0
DOT_NOT_CONVERGED = 1
DOT_EINVAL = -1
DOT_ENOMEM = -2
DOT_EHIP = -3
DOT_EBREAKDOWN = -4
DOT_ENONFINITE = -5

DOT_BC_DIRICHLET = 0
DOT_BC_ROBIN = 1
DOT_FP64 = 0
DOT_MIXED = 1
DOT_PRECOND_AUTO = 0
DOT_PRECOND_JACOBI = 1
DOT_PRECOND_MG = 2
DOT_PRECOND_MG_F32 = 3
DOT_JAC_FP64 = 0
DOT_JAC_SPLIT_BF16 = 1
DOT_JAC_SPLIT_BF16X3 = 2
DOT_ACT_ALPHA = 1
DOT_ACT_BETA = 2
DOT_ACT_CHI = 4
DOT_MAX_COLUMNS = 4096
DOT_NOALLOC_SCRATCH_DOUBLES = 1 << 22
DOT_PROF_PCG1_FP64 = 0
DOT_PROF_PCG2_FP64 = 1
DOT_PROF_PCG1_FP32 = 2
DOT_PROF_PCG2_FP32 = 3
DOT_PROF_RESID = 4
DOT_PROF_JACOBIAN = 5
DOT_PROF_VCYCLE_FP64 = 6
DOT_PROF_VCYCLE_FP32 = 7


class DotGrid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("bc", C.c_int * 6)]


class DotPals(C.Structure):
    _fields_ = [("m0", C.c_int), ("active", C.c_uint), ("mu_in", C.c_double),
                ("mu_out", C.c_double), ("cutoff", C.c_double), ("eps", C.c_double),
                ("gamma", C.c_double)]


class DotSolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int), ("precision", C.c_int),
                ("inner_rtol", C.c_double), ("check_every", C.c_int), ("precond", C.c_int)]


class DotSolveInfo(C.Structure):
    _fields_ = [("iters_max", C.c_int), ("outer", C.c_int),
                ("iters_host", C.POINTER(C.c_int32)), ("relres_host", C.POINTER(C.c_double))]


_vp = C.c_void_p
_i = C.c_int
_d = C.c_double
_sz = C.c_size_t
_i64 = C.c_int64
_pi32 = C.POINTER(C.c_int32)

# name -> (restype, argtypes); every exported function of include/dotpath.h
SIGNATURES = {
    "dot_abi_version": (_i, []),
    "dot_last_error": (C.c_char_p, []),
    "dot_grid_cells": (_i64, [C.POINTER(DotGrid)]),
    "dot_pals_field": (_i, [C.POINTER(DotGrid), C.POINTER(DotPals), _vp, _d, _vp, _vp, _vp]),
    "dot_build_operator": (_i, [C.POINTER(DotGrid), _vp, _vp, C.POINTER(_vp)]),
    "dot_destroy_operator": (_i, [_vp]),
    "dot_operator_cells": (_i64, [_vp]),
    "dot_pals_pairs": (_i64, [_vp]),
    "dot_pals_band_cells": (_i64, [_vp]),
    "dot_set_mua": (_i, [_vp, _vp, _vp]),
    "dot_pals_mua": (_i, [_vp, C.POINTER(DotPals), _vp, _vp, _vp]),
    "dot_pals_mua_diffusion": (_i, [_vp, C.POINTER(DotPals), _d, _d, _vp, _vp, _vp, _vp]),
    "dot_apply": (_i, [_vp, _i, _vp, _vp, _vp]),
    "dot_solve_complex_workspace_bytes": (_sz, [_vp, _i, _i]),
    "dot_solve_complex": (_i, [_vp, _d, _i, _vp, _vp, C.POINTER(DotSolveOpts), _vp, _sz,
                               C.POINTER(DotSolveInfo), _vp]),
    "dot_multigrid_levels": (_i, [_vp]),
    "dot_multigrid_cycle_bytes": (_d, [_vp, _i]),
    "dot_multigrid_workspace_bytes": (_sz, [_vp, _i]),
    "dot_multigrid_apply": (_i, [_vp, _i, _vp, _vp, _vp, _sz, _vp]),
    "dot_form_rhs": (_i, [_vp, _i, _pi32, _i, _vp, _vp, _vp]),
    "dot_solve_workspace_bytes": (_sz, [_vp, _i, _i]),
    "dot_solve_multi_rhs": (_i, [_vp, _i, _i, _vp, _vp, C.POINTER(DotSolveOpts), _vp, _sz,
                                 C.POINTER(DotSolveInfo), _vp]),
    "dot_sampled_misfit": (_i, [_vp, _i, _pi32, _i, _vp, _i, _vp, _vp, _vp,
                                C.POINTER(C.c_double), _vp]),
    "dot_jacobian_workspace_bytes": (_sz, [_vp, _i, _i]),
    "dot_jacobian": (_i, [_vp, _i, _vp, _i, _vp, _i, _vp, _vp, _sz, _vp]),
    "dot_dadp_apply": (_i, [_vp, _i, _vp, _vp, _vp, _vp]),
    "dot_grad_misfit": (_i, [_vp, _i, _vp, _i, _vp, _vp, _vp, _vp, _sz, _vp]),
    "dot_grad_misfit_noalloc": (_i, [_vp, _i, _vp, _i, _vp, _vp, _vp, _vp]),
    "dot_gemm": (_i, [_i, _i, _i, _i, _i, _d, _vp, _i, _vp, _i, _d, _vp, _i, _vp]),
    "dot_mode_gram_workspace_bytes": (_sz, [_i, _i, _i, _i]),
    "dot_mode_gram": (_i, [_i, _i, _i, _vp, _i, _vp, _vp, _sz, _vp]),
    "dot_symeig_workspace_bytes": (_sz, [_i]),
    "dot_symeig": (_i, [_i, _vp, _i, _vp, _vp, _i, _vp, _sz, C.POINTER(C.c_int), _vp]),
    "dot_qr_workspace_bytes": (_sz, [_i, _i]),
    "dot_qr_complete": (_i, [_i, _i, _vp, _i, _vp, _i, _vp, _sz, _vp]),
    "dot_hooi_workspace_bytes": (_sz, [_i, _i, _i, _i, _i]),
    "dot_hooi": (_i, [_i, _i, _i, _vp, _i, _i, _d, _i, _vp, _vp, C.POINTER(C.c_int),
                      C.POINTER(C.c_double), _vp, _sz, _vp]),
    "dot_svd_workspace_bytes": (_sz, [_i, _i]),
    "dot_svd_thin": (_i, [_i, _i, _vp, _i, _vp, _vp, _i, _vp, _i, _d, _vp, _sz, _vp]),
    "dot_tsvd_step_workspace_bytes": (_sz, [_i]),
    "dot_tsvd_step": (_i, [_i, _i, _i, _vp, _i, _vp, _vp, _i, _i, _vp, _vp, _vp, _sz, _vp]),
    "dot_profile_enable": (_i, [_vp, _i]),
    "dot_profile_kinds": (_i, [_vp, C.c_uint]),
    "dot_profile_read": (_i, [_vp, _i, C.POINTER(C.c_double), C.POINTER(_i64),
                              C.POINTER(_i64)]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class DotError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func} failed with code {code}: {msg}")
        self.code = code


class NotConverged(RuntimeWarning):
    pass


def check(code: int, func: str) -> int:
    if code < 0:
        raise DotError(code, func, lib.dot_last_error().decode(errors="replace"))
    return code
