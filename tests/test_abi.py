"""The C-ABI library loads on the CPU and exports every entry point declared in include/pspec.h.

No compute call is made here (there is no GPU); argument validation that returns before any
launch is exercised where it needs no device memory.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pspec.h")
LIB = os.path.join(ROOT, "paper_2605_26975_amd", "libpspec.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pspec_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpspec():
    if not os.path.exists(LIB):
        pytest.fail("libpspec.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("pspec_graph_create", "pspec_objective", "pspec_grad", "pspec_hvp", "pspec_project",
                 "pspec_retract"):
        assert must in names


def test_every_declared_symbol_is_exported(libpspec):
    missing = [n for n in declared_functions() if not hasattr(libpspec, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2605_26975_amd import pspec

    assert sorted(pspec.exported_symbols()) == declared_functions()


def test_host_side_argument_errors(libpspec):
    """Errors found before any launch: NULL output handle, bad sizes, bad k, NULL graph."""
    vp = ctypes.c_void_p
    libpspec.pspec_graph_create.argtypes = [ctypes.c_int64, ctypes.c_int64, vp, vp, vp, ctypes.c_int, ctypes.c_int,
                                            vp, ctypes.POINTER(vp)]
    libpspec.pspec_graph_create.restype = ctypes.c_int
    libpspec.pspec_last_error.restype = ctypes.c_char_p
    h = vp()
    assert libpspec.pspec_graph_create(0, 0, 1, 1, 1, 0, 4, None, ctypes.byref(h)) == 1
    assert b"n = 0" in libpspec.pspec_last_error()
    assert libpspec.pspec_graph_create(10, -1, 1, 1, 1, 0, 4, None, ctypes.byref(h)) == 1
    assert libpspec.pspec_graph_create(10, 5, None, 1, 1, 0, 4, None, ctypes.byref(h)) == 1
    assert libpspec.pspec_graph_create(10, 5, 1, 1, 1, 0, 65, None, ctypes.byref(h)) == 2
    assert libpspec.pspec_graph_create(10, 5, 1, 1, 1, 0, 4, None, None) == 1
    libpspec.pspec_objective.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int64, ctypes.c_double, vp, vp,
                                         vp]
    libpspec.pspec_objective.restype = ctypes.c_int
    assert libpspec.pspec_objective(None, 0, 4, 1, 4, 1.5, None, None, None) == 1
    assert b"NULL graph" in libpspec.pspec_last_error()


def test_dense_argument_errors(libpspec):
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    libpspec.pspec_dense_workspace_bytes.argtypes = [i32]
    libpspec.pspec_dense_workspace_bytes.restype = ctypes.c_size_t
    assert libpspec.pspec_dense_workspace_bytes(16) >= 512 * 16 * 16 * 8
    libpspec.pspec_retract.argtypes = [i64, i32, i32, vp, i64, vp, i64, dbl, vp, i64, vp, vp, ctypes.c_size_t, vp]
    libpspec.pspec_retract.restype = ctypes.c_int
    # n < k, ld < k, k > 64, tiny workspace: all rejected on the host
    assert libpspec.pspec_retract(3, 4, 0, 256, 4, 512, 4, 0.1, 768, 4, None, 1024, 1 << 30, None) == 1
    assert libpspec.pspec_retract(100, 4, 0, 256, 3, 512, 4, 0.1, 768, 4, None, 1024, 1 << 30, None) == 1
    assert libpspec.pspec_retract(100, 65, 0, 256, 65, 512, 65, 0.1, 768, 65, None, 1024, 1 << 30, None) == 2
    assert libpspec.pspec_retract(100, 4, 0, 256, 4, 512, 4, 0.1, 768, 4, None, 1024, 16, None) == 4


def test_rhvp_host_side_errors(libpspec):
    """pspec_rhvp rejects a NULL graph before any launch, and the dense workspace covers the two
    k x k partials per Gram workgroup it needs."""
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    libpspec.pspec_rhvp.argtypes = [vp, i32, i32, vp, i64, vp, i64, dbl, dbl, vp, i64, vp, i64, vp, vp, vp,
                                    ctypes.c_size_t, vp]
    libpspec.pspec_rhvp.restype = ctypes.c_int
    libpspec.pspec_last_error.restype = ctypes.c_char_p
    assert libpspec.pspec_rhvp(None, 0, 16, 256, 32, 320, 32, 1.5, 1e-8, 512, 16, 768, 16, None, None, 1024,
                               1 << 30, None) == 1
    assert b"rhvp: NULL graph" in libpspec.pspec_last_error()
    libpspec.pspec_dense_workspace_bytes.argtypes = [i32]
    libpspec.pspec_dense_workspace_bytes.restype = ctypes.c_size_t
    assert libpspec.pspec_dense_workspace_bytes(16) >= 2 * 1024 * 16 * 16 * 8


def test_kmeans_host_side_errors(libpspec):
    """pspec_kmeans_step validates sizes, pointers and the workspace on the host, before any launch;
    the workspace covers one c x (d + 2) partial per workgroup."""
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    libpspec.pspec_kmeans_step.argtypes = [i64, i32, i32, vp, i64, i32, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    libpspec.pspec_kmeans_step.restype = ctypes.c_int
    libpspec.pspec_kmeans_workspace_bytes.argtypes = [i32, i32]
    libpspec.pspec_kmeans_workspace_bytes.restype = ctypes.c_size_t
    libpspec.pspec_last_error.restype = ctypes.c_char_p
    ws = libpspec.pspec_kmeans_workspace_bytes(4, 4)
    assert ws >= 1024 * 4 * 6 * 8
    call = libpspec.pspec_kmeans_step
    # (n, d, dt, X, ldx, c, C, labels, dist, stats, ws, ws_bytes, stream)
    assert call(-1, 4, 0, 256, 4, 4, 512, None, None, 768, 1024, ws, None) == 1
    assert call(100, 0, 0, 256, 4, 4, 512, None, None, 768, 1024, ws, None) == 1
    assert call(100, 33, 0, 256, 33, 4, 512, None, None, 768, 1024, 1 << 30, None) == 2
    assert call(100, 4, 0, 256, 4, 0, 512, None, None, 768, 1024, ws, None) == 1
    assert call(100, 4, 0, 256, 4, 33, 512, None, None, 768, 1024, 1 << 30, None) == 2
    assert call(100, 4, 0, 256, 3, 4, 512, None, None, 768, 1024, ws, None) == 1
    assert b"ldx" in libpspec.pspec_last_error()
    assert call(100, 4, 0, None, 4, 4, 512, None, None, 768, 1024, ws, None) == 1
    assert call(100, 4, 0, 256, 4, 4, None, None, None, 768, 1024, ws, None) == 1
    assert call(100, 4, 0, 256, 4, 4, 512, None, None, None, 1024, ws, None) == 1
    assert call(100, 4, 0, 256, 4, 4, 512, None, None, 768, 1000, ws, None) == 1
    assert call(100, 4, 0, 256, 4, 4, 512, None, None, 768, 1024, ws - 8, None) == 4
    assert b"workspace" in libpspec.pspec_last_error()
