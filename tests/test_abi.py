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
    sz = ctypes.c_size_t
    libpspec.pspec_graph_create.argtypes = [ctypes.c_int64, ctypes.c_int64, vp, vp, vp, ctypes.c_int, ctypes.c_int,
                                            vp, sz, vp, ctypes.POINTER(vp)]
    libpspec.pspec_graph_create.restype = ctypes.c_int
    libpspec.pspec_graph_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
    libpspec.pspec_graph_workspace_bytes.restype = sz
    libpspec.pspec_last_error.restype = ctypes.c_char_p
    h = vp()
    ws, big = 1 << 20, 1 << 40  # a 256-aligned stand-in address: nothing is dereferenced on these paths
    assert libpspec.pspec_graph_create(0, 0, 1, 1, 1, 0, 4, ws, big, None, ctypes.byref(h)) == 1
    assert b"n = 0" in libpspec.pspec_last_error()
    assert libpspec.pspec_graph_create(10, -1, 1, 1, 1, 0, 4, ws, big, None, ctypes.byref(h)) == 1
    assert libpspec.pspec_graph_create(10, 5, None, 1, 1, 0, 4, ws, big, None, ctypes.byref(h)) == 1
    assert libpspec.pspec_graph_create(10, 5, 1, 1, 1, 0, 65, ws, big, None, ctypes.byref(h)) == 2
    assert libpspec.pspec_graph_create(10, 5, 1, 1, 1, 0, 4, ws, big, None, None) == 1
    assert libpspec.pspec_graph_create(10, 5, 1, 1, 1, 0, 4, None, big, None, ctypes.byref(h)) == 1
    assert libpspec.pspec_graph_create(10, 5, 1, 1, 1, 0, 4, ws + 8, big, None, ctypes.byref(h)) == 1
    assert b"aligned" in libpspec.pspec_last_error()
    # below the counting part: refused before any device access (ws is not a device address)
    libpspec.pspec_graph_count_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int]
    libpspec.pspec_graph_count_workspace_bytes.restype = sz
    fixed = libpspec.pspec_graph_count_workspace_bytes(10, 4)
    assert 0 < fixed <= libpspec.pspec_graph_workspace_bytes(10, 5, 4) < libpspec.pspec_graph_workspace_bytes(10, 5000, 4)
    assert libpspec.pspec_graph_create(10, 5, 1, 1, 1, 0, 4, ws, fixed - 1, None, ctypes.byref(h)) == 4
    libpspec.pspec_graph_exact_workspace.argtypes = [ctypes.c_int64, ctypes.c_int64, vp, vp, ctypes.c_int, vp, sz,
                                                     vp, ctypes.POINTER(sz)]
    libpspec.pspec_graph_exact_workspace.restype = ctypes.c_int
    need = sz()
    assert libpspec.pspec_graph_exact_workspace(10, 5, 1, 1, 4, ws, fixed - 1, None, ctypes.byref(need)) == 4
    assert libpspec.pspec_graph_exact_workspace(10, 5, 1, 1, 4, ws, fixed, None, None) == 1
    assert libpspec.pspec_graph_workspace_bytes(0, 5, 4) == 0 and libpspec.pspec_graph_workspace_bytes(10, 5, 65) == 0
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


def test_graph_workspace_bound_covers_every_schedule():
    """pspec_graph_workspace_bytes bounds the schedule from (n, nnz, k_max) alone: it grows with each
    and covers the worst degree patterns (every row just above the light limit, one giant row)."""
    lib = ctypes.CDLL(LIB)
    f = lib.pspec_graph_workspace_bytes
    f.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
    f.restype = ctypes.c_size_t
    n, nnz = 1000, 33 * 1000
    chunk, light = 512, 32
    base = f(n, nnz, 8)
    assert f(n, nnz, 16) > base and f(n, 2 * nnz, 8) > base and f(2 * n, nnz, 8) > base
    # all rows of degree 33: 1000 heavy rows, 1000 chunks of 24 bytes; one row of degree 33000: 65 chunks,
    # all of them split chunks with 2 k_max doubles of scratch each
    # one row of degree 33000 cut at 8 segment boundaries: at most 65 + 8 chunks, all split chunks
    worst_chunks = max(n, -(-nnz // chunk) + 8)
    assert base >= 24 * worst_chunks + 2 * 8 * 8 * (-(-nnz // chunk) + 8)
    assert f(n, 0, 8) > 0  # an empty graph still needs its partial sums
    # k_max > 8 adds the Gram area of the Riemannian call (one 4 x 16 x 16 FP64 partial per 256-row
    # tile and per heavy-row workgroup, plus the rows of its fixed-order reduction)
    assert f(n, nnz, 9) - f(n, nnz, 8) >= 8192 * (-(-n // 256) + 256 + 1024 + 32 + 1)


def test_binding_rejects_mismatched_blocks(monkeypatch):
    """The binding is the guard in front of a pointer-only ABI: every block must have the graph's n
    rows, the same k, dtype and device, and scalar outputs the right size, before any call is made.
    Exercised with host tensors standing in for device ones (the checks raise before the library is
    reached, so no GPU is needed)."""
    import torch

    from paper_2605_26975_amd import pspec

    monkeypatch.setattr(pspec, "_on_device", lambda t: isinstance(t, torch.Tensor))

    class FakeGraph:
        n, k_max, device = 100, 8, torch.device("cpu")
        handle = None

    g = FakeGraph()
    U = torch.zeros(100, 8)
    bad = {
        "short U": lambda: pspec.objective(g, torch.zeros(99, 8), 1.5),
        "k above k_max": lambda: pspec.objective(g, torch.zeros(100, 9), 1.5),
        "short V": lambda: pspec.hvp(g, U, torch.zeros(99, 8), 1.5),
        "V with other k": lambda: pspec.hvp(g, U, torch.zeros(100, 7), 1.5),
        "V float64": lambda: pspec.hvp(g, U, torch.zeros(100, 8, dtype=torch.float64), 1.5),
        "short G": lambda: pspec.grad(g, U, 1.5, G=torch.zeros(50, 8)),
        "HV float64": lambda: pspec.hvp(g, U, U.clone(), 1.5, HV=torch.zeros(100, 8, dtype=torch.float64)),
        "F_col too short": lambda: pspec.hvp(g, U, U.clone(), 1.5, F_col=torch.zeros(7, dtype=torch.float64)),
        "F_col float32": lambda: pspec.objective(g, U, 1.5, F_col=torch.zeros(8)),
        "RH short": lambda: pspec.rhvp(g, U, U.clone(), 1.5, RH=torch.zeros(10, 8)),
        "MG wrong size": lambda: pspec.rhvp(g, U, U.clone(), 1.5, MG=torch.zeros(4, 4, dtype=torch.float64)),
        "Z other k": lambda: pspec.project(U, torch.zeros(100, 4)),
        "X without MX": lambda: pspec.project(U, U.clone(), X=U.clone()),
        "out short": lambda: pspec.project(U, U.clone(), out=torch.zeros(100, 4)),
        "eta float64": lambda: pspec.retract(U, torch.zeros(100, 8, dtype=torch.float64), 0.1),
        "dot mismatch": lambda: pspec.dot(U, torch.zeros(100, 9)),
        "axpby mismatch": lambda: pspec.axpby(1.0, torch.zeros(90, 8), 0.0, U),
        "int block": lambda: pspec.dot(torch.zeros(100, 8, dtype=torch.int32), torch.zeros(100, 8, dtype=torch.int32)),
        "overlapping rows": lambda: pspec.dot(torch.zeros(800).as_strided((100, 8), (4, 1)), U),
        "column-major": lambda: pspec.dot(torch.zeros(8, 100).t(), U),
    }
    for what, call in bad.items():
        with pytest.raises(pspec.PSpecArgError):
            call()
            pytest.fail(what)
