"""CPU-side checks of the C ABI: the library loads, exports every function that
include/dotpath.h declares, and rejects invalid arguments on the host before
any HIP call (so these run without a GPU)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dotpath.h")


def _header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dot_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_1706_05586_amd import _lib
    return _lib


def test_every_declared_symbol_is_exported(L):
    names = _header_functions()
    assert len(names) >= 15
    raw = C.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), f"{n} declared in dotpath.h but not exported"
    # and the binding declares exactly the header's functions
    assert set(L.SIGNATURES) == set(names)


def test_abi_version(L):
    assert L.lib.dot_abi_version() == 2


def _grid(L, dim=3, n=(8, 8, 8), bc=(0, 0, 0, 0, 1, 1)):
    g = L.DotGrid()
    g.dim = dim
    for a in range(3):
        g.n[a] = n[a] if a < len(n) else 1
    for f in range(6):
        g.bc[f] = bc[f] if f < len(bc) else 0
    return g


def test_grid_validation(L):
    assert L.lib.dot_grid_cells(C.byref(_grid(L))) == 512
    assert L.lib.dot_grid_cells(C.byref(_grid(L, dim=2, n=(5, 7, 99)))) == 35
    assert L.lib.dot_grid_cells(C.byref(_grid(L, dim=4))) == -1
    assert L.lib.dot_grid_cells(C.byref(_grid(L, n=(0, 8, 8)))) == -1
    assert L.lib.dot_grid_cells(C.byref(_grid(L, bc=(0, 0, 2, 0, 1, 1)))) == -1
    assert L.lib.dot_grid_cells(None) == -1


def test_invalid_arguments_rejected_before_hip(L):
    g = _grid(L, dim=5)
    out = C.c_void_p()
    rc = L.lib.dot_build_operator(C.byref(g), C.c_void_p(1), None, C.byref(out))
    assert rc == L.DOT_EINVAL and b"dim" in L.lib.dot_last_error()
    rc = L.lib.dot_build_operator(C.byref(_grid(L)), None, None, C.byref(out))
    assert rc == L.DOT_EINVAL
    # NULL handle everywhere
    assert L.lib.dot_set_mua(None, C.c_void_p(1), None) == L.DOT_EINVAL
    assert L.lib.dot_apply(None, 1, C.c_void_p(1), C.c_void_p(2), None) == L.DOT_EINVAL
    opts = L.DotSolveOpts(1e-8, 100, 0, 0.1, 8)
    assert L.lib.dot_solve_multi_rhs(None, 0, 1, C.c_void_p(1), C.c_void_p(2), C.byref(opts),
                                     None, 0, None, None) == L.DOT_EINVAL
    assert L.lib.dot_jacobian(None, 1, None, 1, None, 0, None, None, 0, None) == L.DOT_EINVAL
    assert L.lib.dot_grad_misfit(None, 1, None, 1, None, None, None, None, 0, None) == L.DOT_EINVAL
    assert L.lib.dot_solve_workspace_bytes(None, 4, 0) == 0
    assert L.lib.dot_jacobian_workspace_bytes(None, 4, 4) == 0
    cells = np.zeros(1, dtype=np.int32)
    f = C.c_double()
    assert L.lib.dot_sampled_misfit(None, 1, cells.ctypes.data_as(L._pi32), 1, None, 1, None,
                                    None, None, C.byref(f), None) == L.DOT_EINVAL
    assert L.lib.dot_gemm(0, 0, -1, 1, 1, 1.0, None, 1, None, 1, 0.0, None, 1, None) == L.DOT_EINVAL
    # a zero-size product is a no-op
    assert L.lib.dot_gemm(0, 0, 0, 3, 3, 1.0, None, 1, None, 3, 0.0, None, 1, None) == L.DOT_OK


def test_pals_descriptor_validation(L):
    g = _grid(L)
    p = L.DotPals(0, 7, 0.05, 0.01, 0.15, 0.1, 1e-3)
    assert L.lib.dot_pals_field(C.byref(g), C.byref(p), C.c_void_p(1), 1.0, C.c_void_p(2), None,
                                None) == L.DOT_EINVAL
    p = L.DotPals(4, 8, 0.05, 0.01, 0.15, 0.1, 1e-3)
    assert L.lib.dot_pals_field(C.byref(g), C.byref(p), C.c_void_p(1), 1.0, C.c_void_p(2), None,
                                None) == L.DOT_EINVAL
    p = L.DotPals(4, 7, 0.05, 0.01, 0.15, -0.1, 1e-3)
    assert L.lib.dot_pals_field(C.byref(g), C.byref(p), C.c_void_p(1), 1.0, C.c_void_p(2), None,
                                None) == L.DOT_EINVAL
    p = L.DotPals(4, 7, 0.05, 0.01, 0.15, 0.1, 1e-3)
    assert L.lib.dot_pals_field(C.byref(g), C.byref(p), None, 1.0, C.c_void_p(2), None,
                                None) == L.DOT_EINVAL


def test_product_path_has_no_oracle_dependency():
    pkg = os.path.join(ROOT, "paper_1706_05586_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn


def test_grid_cell_cap(L):
    """The sweeps address one binary64 column with 32-bit byte offsets: grids
    of more than 2^29 cells are refused on the host."""
    assert L.lib.dot_grid_cells(C.byref(_grid(L, n=(1024, 1024, 512)))) == 1 << 29
    assert L.lib.dot_grid_cells(C.byref(_grid(L, n=(1024, 1024, 513)))) == -1
    out = C.c_void_p()
    rc = L.lib.dot_build_operator(C.byref(_grid(L, n=(1024, 1024, 513))), C.c_void_p(1), None,
                                  C.byref(out))
    assert rc == L.DOT_EINVAL and b"2^29" in L.lib.dot_last_error()


def test_output_block_checks():
    """Caller-supplied output blocks (solve's out, form_rhs's out) are checked
    for shape, dtype and column-major layout before the library writes them."""
    import torch

    from paper_1706_05586_amd.api import check_field_block
    good = torch.empty((3, 10), dtype=torch.float64).t()          # (10, 3) column-major
    with pytest.raises(ValueError, match="shape"):
        check_field_block(good[:9], 10, 3)
    with pytest.raises(TypeError, match="float64"):
        check_field_block(torch.empty((3, 10), dtype=torch.float32).t(), 10, 3)
    with pytest.raises(ValueError, match="column-major"):
        check_field_block(torch.empty((10, 3), dtype=torch.float64), 10, 3)
    with pytest.raises(TypeError, match="CUDA"):
        check_field_block(good, 10, 3)   # layout right, but host memory
    # a column slice of a column-major block is itself column-major
    with pytest.raises(TypeError, match="CUDA"):
        check_field_block(good[:, 1:], 10, 2)
