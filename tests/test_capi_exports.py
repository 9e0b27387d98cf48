"""The C-ABI library loads on any machine and exports every function include/qcpd.h
declares; the ctypes structures match the header's layout."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qcpd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qcpd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2508_17522_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(_capi.LIB_PATH)
    names = declared_functions()
    assert "qcpd_create" in names and "qcpd_jvp" in names and "qcpd_vjp" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(_capi.EXPORTS) == names


def test_struct_layouts():
    from paper_2508_17522_amd import _capi as C
    assert ctypes.sizeof(C.qcpd_csr) == 4 * 3 + 4 + 8 * 3  # 3 int32 + padding + 3 pointers
    assert ctypes.sizeof(C.qcpd_opts) == 8 + 4 * 15 + 4  # 15 int32 fields, tail padding
    assert ctypes.sizeof(C.qcpd_info) == 4 + 4 + 8 + 8 + 4 + 4


def test_status_strings_without_gpu():
    from paper_2508_17522_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        pytest.skip("library not built")
    lib = _capi.load()
    assert lib.qcpd_status_str(0) == b"ok"
    assert b"NaN" in lib.qcpd_status_str(-5)


def test_default_options_without_gpu():
    """qcpd_opts_default fills every field: the documented defaults, and 0 (the library's
    choice) in each launch-layout field, whatever the caller's struct held before."""
    from paper_2508_17522_amd import _capi as C
    if not os.path.exists(C.LIB_PATH):
        pytest.skip("library not built")
    lib = C.load()
    o = C.qcpd_opts()
    ctypes.memset(ctypes.byref(o), 0x5A, ctypes.sizeof(o))
    lib.qcpd_opts_default(ctypes.byref(o))
    assert (o.tol, o.max_iter, o.precond, o.graph_chunk, o.check_symmetry, o.engine,
            o.solver) == (1e-8, 0, C.QCPD_PRECOND_JACOBI, 128, 1, C.QCPD_ENGINE_AUTO,
                          C.QCPD_SOLVER_LSQR)
    for name in ("staged", "deep", "nnz_per_lane_F", "nnz_per_lane_FT", "lanes_x", "lanes_y",
                 "loop_grid", "persist_grid", "equil_sweeps"):
        assert getattr(o, name) == 0, name
