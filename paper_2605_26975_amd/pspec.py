"""ctypes binding of libpspec.so (C ABI in include/pspec.h).

Argument marshalling only: every computation runs in the HIP library.  Torch supplies device
memory (tensor data pointers) and streams (the current stream of the tensor's device).  The
library must be built (``python -m paper_2605_26975_amd.build``); if it is missing, every call
raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

# The in-tree build; PSPEC_LIBRARY may name another build of the same C ABI.
LIB_PATH = os.environ.get("PSPEC_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpspec.so")

PSPEC_F32, PSPEC_F64 = 0, 1
_STATUS = {0: "PSPEC_OK", 1: "PSPEC_ERR_ARG", 2: "PSPEC_ERR_UNSUPPORTED", 3: "PSPEC_ERR_HIP", 4: "PSPEC_ERR_WORKSPACE"}
LIGHT_MAX = 32
CHUNK = 512
K_MAX = 64

_lib = None


class PSpecError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class PSpecArgError(PSpecError, ValueError, TypeError):
    """An argument the binding rejects before calling the library (status PSPEC_ERR_ARG): a tensor
    of the wrong shape, dtype, device or layout.  Also a ValueError and a TypeError."""

    def __init__(self, msg: str):
        super().__init__(1, msg)


def lib() -> ctypes.CDLL:
    """Load libpspec.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2605_26975_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    sig = {
        "pspec_graph_create": [i64, i64, vp, vp, vp, i32, i32, vp, sz, vp, ctypes.POINTER(vp)],
        "pspec_graph_destroy": [vp],
        "pspec_graph_info": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "pspec_graph_ascending": [vp, ctypes.POINTER(i32)],
        "pspec_graph_degree_order": [vp, ctypes.POINTER(i32)],
        "pspec_graph_set_timing_events": [vp, vp, vp],
        "pspec_objective": [vp, i32, i32, vp, i64, dbl, vp, vp, vp],
        "pspec_grad": [vp, i32, i32, vp, i64, dbl, vp, i64, vp, vp],
        "pspec_hvp": [vp, i32, i32, vp, i64, vp, i64, dbl, dbl, vp, i64, vp, i64, vp, vp],
        "pspec_hvp_sparse": [vp, i32, i32, vp, i64, vp, i64, dbl, dbl, vp, i64, vp, i64, vp, vp],
        "pspec_hvp_gather_floor": [vp, i32, vp, i64, vp, i64, vp, i64, vp, i64, vp],
        "pspec_rhvp": [vp, i32, i32, vp, i64, vp, i64, dbl, dbl, vp, i64, vp, i64, vp, vp, vp, sz, vp],
        "pspec_rhvp_static": [vp, i32, i32, vp, i64, vp, i64, dbl, dbl, vp, i64, vp, i64, vp, vp, vp],
        "pspec_rhess": [vp, i32, i32, vp, i64, vp, i64, vp, i64, dbl, dbl, vp, i64, vp, vp, vp, sz, vp],
        "pspec_project": [i64, i32, i32, vp, i64, vp, i64, vp, i64, vp, vp, i64, vp, vp, sz, vp],
        "pspec_retract": [i64, i32, i32, vp, i64, vp, i64, dbl, vp, i64, vp, vp, sz, vp],
        "pspec_dot": [i64, i32, i32, vp, i64, vp, i64, vp, vp, sz, vp],
        "pspec_axpby": [i64, i32, i32, dbl, vp, i64, dbl, vp, i64, vp],
        "pspec_kmeans_step": [i64, i32, i32, vp, i64, i32, vp, vp, vp, vp, vp, sz, vp],
        "pspec_rcm_order": [i64, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.pspec_graph_workspace_bytes.argtypes = [i64, i64, i32]
    L.pspec_graph_workspace_bytes.restype = sz
    L.pspec_graph_count_workspace_bytes.argtypes = [i64, i32]
    L.pspec_graph_count_workspace_bytes.restype = sz
    L.pspec_graph_exact_workspace.argtypes = [i64, i64, vp, vp, i32, vp, sz, vp, ctypes.POINTER(sz)]
    L.pspec_graph_exact_workspace.restype = ctypes.c_int
    L.pspec_dense_workspace_bytes.argtypes = [i32]
    L.pspec_dense_workspace_bytes.restype = sz
    L.pspec_kmeans_workspace_bytes.argtypes = [i32, i32]
    L.pspec_kmeans_workspace_bytes.restype = sz
    L.pspec_last_error.argtypes = []
    L.pspec_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def exported_symbols() -> list[str]:
    """Names of the entry points the binding declares (all must resolve in the library)."""
    return [
        "pspec_graph_workspace_bytes", "pspec_graph_count_workspace_bytes", "pspec_graph_exact_workspace",
        "pspec_graph_create", "pspec_graph_destroy", "pspec_graph_info", "pspec_graph_ascending",
        "pspec_graph_degree_order",
        "pspec_graph_set_timing_events",
        "pspec_objective", "pspec_grad",
        "pspec_hvp", "pspec_hvp_sparse", "pspec_hvp_gather_floor", "pspec_rhvp", "pspec_rhvp_static", "pspec_rhess", "pspec_dense_workspace_bytes", "pspec_project", "pspec_retract", "pspec_dot",
        "pspec_axpby", "pspec_kmeans_workspace_bytes", "pspec_kmeans_step", "pspec_rcm_order",
        "pspec_last_error",
    ]


def _check(status: int) -> None:
    if status != 0:
        raise PSpecError(status, lib().pspec_last_error().decode())


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return PSPEC_F32
    if t.dtype == torch.float64:
        return PSPEC_F64
    raise PSpecArgError(f"unsupported dtype {t.dtype}")


def _on_device(t) -> bool:
    return isinstance(t, torch.Tensor) and t.is_cuda


def _block(t: torch.Tensor, name: str, like: torch.Tensor | None = None, n: int | None = None) -> int:
    """Validate an n x k row-major device block; return its leading dimension.  With ``like`` the
    block must also have like's shape, dtype and device; with ``n`` exactly n rows.  The C ABI takes
    bare pointers and sizes every access from n and k, so a short or mismatched block would be read
    or written out of bounds: every mismatch raises here, before anything is launched."""
    if not _on_device(t):
        raise PSpecArgError(f"{name} must be a device tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise PSpecArgError(f"{name} must be 2-D with unit column stride (row-major)")
    if t.dtype not in (torch.float32, torch.float64):
        raise PSpecArgError(f"{name} must be float32 or float64, not {t.dtype}")
    if t.shape[0] > 1 and t.stride(0) < t.shape[1]:
        raise PSpecArgError(f"{name}: rows overlap (leading dimension {t.stride(0)} < {t.shape[1]} columns)")
    if like is not None:
        if tuple(t.shape) != tuple(like.shape):
            raise PSpecArgError(f"{name} has shape {tuple(t.shape)}, expected {tuple(like.shape)}")
        if t.dtype != like.dtype:
            raise PSpecArgError(f"{name} has dtype {t.dtype}, expected {like.dtype}")
        if t.device != like.device:
            raise PSpecArgError(f"{name} is on {t.device}, expected {like.device}")
    if n is not None and t.shape[0] != n:
        raise PSpecArgError(f"{name} has {t.shape[0]} rows, the graph has {n} nodes")
    return t.stride(0)


def _fp64_vec(t: torch.Tensor, name: str, size: int, device) -> None:
    """A contiguous float64 device tensor of ``size`` elements (scalar outputs)."""
    if not (_on_device(t) and t.dtype == torch.float64 and t.is_contiguous()
            and t.numel() == size and t.device == torch.device(device)):
        raise PSpecArgError(f"{name} must be a contiguous float64 tensor of {size} elements on {device}")


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


# Workspaces of the dense calls, one per (device, stream, kind): the library requires that a
# workspace is used by one call at a time, and calls on one stream run one after another.
_ws_cache: dict = {}


def _dense_ws(device, k: int) -> torch.Tensor:
    nbytes = int(lib().pspec_dense_workspace_bytes(k))
    key = (str(device), _stream(device), k)
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        _ws_cache[key] = ws
    return ws


class Graph:
    """A device CSR graph with its row schedule (pspec_graph_create).  Keeps the CSR tensors and the
    schedule's workspace (a torch buffer of pspec_graph_workspace_bytes bytes) alive."""

    def __init__(self, rowptr: torch.Tensor, col: torch.Tensor, w: torch.Tensor, k_max: int):
        for t, name, dt in ((rowptr, "rowptr", torch.int64), (col, "col", torch.int32)):
            if not t.is_cuda or t.dtype != dt or t.dim() != 1 or not t.is_contiguous():
                raise PSpecArgError(f"{name} must be a contiguous 1-D {dt} device tensor")
        if not w.is_cuda or w.dim() != 1 or not w.is_contiguous():
            raise PSpecArgError("w must be a contiguous 1-D device tensor")
        if col.device != rowptr.device or w.device != rowptr.device:
            raise PSpecArgError("rowptr, col and w must be on one device")
        if w.numel() != col.numel():
            raise PSpecArgError(f"w has {w.numel()} entries, col {col.numel()}")
        self.rowptr, self.col, self.w = rowptr, col, w
        self.n = rowptr.numel() - 1
        self.nnz = col.numel()
        self.k_max = k_max
        self.device = rowptr.device
        self._h = ctypes.c_void_p()
        if int(lib().pspec_graph_workspace_bytes(self.n, self.nnz, k_max)) == 0:
            raise PSpecArgError(f"graph_create: n = {self.n}, nnz = {self.nnz}, k_max = {k_max} rejected")
        with torch.cuda.device(self.device):
            # exact sizing: count the schedule in the fixed part, then grow the buffer to what it needs
            nfix = int(lib().pspec_graph_count_workspace_bytes(self.n, k_max))
            tmp = torch.empty(nfix, dtype=torch.uint8, device=self.device)
            need = ctypes.c_size_t()
            _check(lib().pspec_graph_exact_workspace(self.n, self.nnz, rowptr.data_ptr(), col.data_ptr(), k_max,
                                                     tmp.data_ptr(), nfix, _stream(self.device), ctypes.byref(need)))
            del tmp
            self.workspace = torch.empty(need.value, dtype=torch.uint8, device=self.device)
            _check(lib().pspec_graph_create(self.n, self.nnz, rowptr.data_ptr(), col.data_ptr(), w.data_ptr(),
                                            _dtype_code(w), k_max, self.workspace.data_ptr(), need.value,
                                            _stream(self.device), ctypes.byref(self._h)))

    @classmethod
    def from_host(cls, g, device="cuda", k_max: int = K_MAX, weight_dtype=torch.float32) -> "Graph":
        """From any object with numpy rowptr/col/w (e.g. paper_2605_26975_amd.gen.Graph)."""
        rowptr = torch.as_tensor(g.rowptr, dtype=torch.int64).to(device)
        col = torch.as_tensor(g.col, dtype=torch.int32).to(device)
        w = torch.as_tensor(g.w).to(weight_dtype).to(device)
        return cls(rowptr, col, w, k_max)

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("graph is closed")
        return self._h

    def info(self) -> dict:
        h, c, s = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().pspec_graph_info(self.handle, ctypes.byref(h), ctypes.byref(c), ctypes.byref(s)))
        a, o = ctypes.c_int(), ctypes.c_int()
        _check(lib().pspec_graph_ascending(self.handle, ctypes.byref(a)))
        _check(lib().pspec_graph_degree_order(self.handle, ctypes.byref(o)))
        return dict(heavy_rows=h.value, chunks=c.value, split_rows=s.value, ascending=bool(a.value),
                    degree_order=bool(o.value))

    def set_timing_events_raw(self, before, after) -> None:
        """Record two raw hipEvent_t handles (or None, None) around the edge pass of later calls."""
        _check(lib().pspec_graph_set_timing_events(self.handle, before, after))

    def close(self) -> None:
        """Release the handle (no synchronisation).  The workspace tensor is returned to torch's
        allocator, which orders its reuse after the work already enqueued on this stream."""
        if self._h:
            _check(lib().pspec_graph_destroy(self._h))
            self._h = ctypes.c_void_p()
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _on_graph(graph: Graph, U: torch.Tensor) -> int:
    """Checks shared by the edge-pass calls; returns U's leading dimension."""
    ldu = _block(U, "U", n=graph.n)
    if U.device != graph.device:
        raise PSpecArgError(f"U is on {U.device}, the graph on {graph.device}")
    if not 1 <= U.shape[1] <= graph.k_max:
        raise PSpecArgError(f"U has {U.shape[1]} columns; the graph was built for 1..{graph.k_max}")
    return ldu


def _out_block(t: torch.Tensor | None, name: str, like: torch.Tensor) -> torch.Tensor:
    """An output block: a new n x k tensor like ``like``, or a caller tensor checked against it."""
    if t is None:
        return torch.empty(like.shape, dtype=like.dtype, device=like.device)
    _block(t, name, like=like)
    return t


def _fcol(F_col, k, device):
    if F_col is None:
        return torch.empty(k, dtype=torch.float64, device=device)
    _fp64_vec(F_col, "F_col", k, device)
    return F_col


def objective(graph: Graph, U: torch.Tensor, p: float, F_col: torch.Tensor | None = None,
              F: torch.Tensor | None = None):
    """Eq. (1): returns (F, F_col) as FP64 device tensors (0-dim and k)."""
    ldu = _on_graph(graph, U)
    k = U.shape[1]
    F_col = _fcol(F_col, k, U.device)
    if F is None:
        F = torch.empty((), dtype=torch.float64, device=U.device)
    _fp64_vec(F, "F", 1, U.device)
    _check(lib().pspec_objective(graph.handle, _dtype_code(U), k, U.data_ptr(), ldu, float(p), F_col.data_ptr(),
                                 F.data_ptr(), _stream(U.device)))
    return F, F_col


def grad(graph: Graph, U: torch.Tensor, p: float, G: torch.Tensor | None = None, F_col: torch.Tensor | None = None):
    """Euclidean gradient of Eq. (1): returns (G, F_col)."""
    ldu = _on_graph(graph, U)
    k = U.shape[1]
    G = _out_block(G, "G", U)
    F_col = _fcol(F_col, k, U.device)
    _check(lib().pspec_grad(graph.handle, _dtype_code(U), k, U.data_ptr(), ldu, float(p), G.data_ptr(),
                            G.stride(0), F_col.data_ptr(), _stream(U.device)))
    return G, F_col


def hvp(graph: Graph, U: torch.Tensor, V: torch.Tensor, p: float, eps: float = 1e-8,
        HV: torch.Tensor | None = None, G: torch.Tensor | None = None, F_col: torch.Tensor | None = None,
        sparse_only: bool = False):
    """Hessian of Eq. (1) at U applied to V, fused with the gradient: returns (HV, G, F_col).
    ``sparse_only`` drops the dense rank-2 part of the Hessian (pspec_hvp_sparse)."""
    ldu = _on_graph(graph, U)
    ldv = _block(V, "V", like=U)
    k = U.shape[1]
    HV = _out_block(HV, "HV", U)
    G = _out_block(G, "G", U)
    F_col = _fcol(F_col, k, U.device)
    fn = lib().pspec_hvp_sparse if sparse_only else lib().pspec_hvp
    _check(fn(graph.handle, _dtype_code(U), k, U.data_ptr(), ldu, V.data_ptr(), ldv, float(p), float(eps),
              HV.data_ptr(), HV.stride(0), G.data_ptr(), G.stride(0), F_col.data_ptr(), _stream(U.device)))
    return HV, G, F_col


def hvp_gather_floor(graph: Graph, U: torch.Tensor, V: torch.Tensor, HV: torch.Tensor | None = None,
                     G: torch.Tensor | None = None):
    """Measurement reference (not the method): the FP32 HVP edge pass with its arithmetic replaced by
    a sum of the gathered values (pspec_hvp_gather_floor).  Returns (HV, G) with meaningless values."""
    ldu = _on_graph(graph, U)
    ldv = _block(V, "V", like=U)
    if U.dtype != torch.float32:
        raise PSpecArgError("hvp_gather_floor runs on float32 blocks")
    HV = _out_block(HV, "HV", U)
    G = _out_block(G, "G", U)
    _check(lib().pspec_hvp_gather_floor(graph.handle, U.shape[1], U.data_ptr(), ldu, V.data_ptr(), ldv,
                                        HV.data_ptr(), HV.stride(0), G.data_ptr(), G.stride(0), _stream(U.device)))
    return HV, G


def rhvp(graph: Graph, U: torch.Tensor, V: torch.Tensor, p: float, eps: float = 1e-8,
         RH: torch.Tensor | None = None, RG: torch.Tensor | None = None, MG: torch.Tensor | None = None,
         F_col: torch.Tensor | None = None):
    """Riemannian Hessian at U applied to the tangent vector V and Riemannian gradient, fused:
    returns (RH = P_U(H V) - V (U^T G), RG = P_U(G), MG = U^T G, F_col)."""
    ldu = _on_graph(graph, U)
    ldv = _block(V, "V", like=U)
    k = U.shape[1]
    RH = _out_block(RH, "RH", U)
    RG = _out_block(RG, "RG", U)
    if MG is None:
        MG = torch.empty((k, k), dtype=torch.float64, device=U.device)
    _fp64_vec(MG, "MG", k * k, U.device)
    F_col = _fcol(F_col, k, U.device)
    ws = _dense_ws(U.device, k)
    _check(lib().pspec_rhvp(graph.handle, _dtype_code(U), k, U.data_ptr(), ldu, V.data_ptr(), ldv, float(p),
                            float(eps), RH.data_ptr(), RH.stride(0), RG.data_ptr(), RG.stride(0),
                            MG.data_ptr(), F_col.data_ptr(), ws.data_ptr(), ws.numel(), _stream(U.device)))
    return RH, RG, MG, F_col


def rhess(graph: Graph, U: torch.Tensor, V: torch.Tensor, G: torch.Tensor, p: float, eps: float = 1e-8,
          RH: torch.Tensor | None = None, MG: torch.Tensor | None = None, F_col: torch.Tensor | None = None):
    """Riemannian Hessian at U applied to the tangent vector V, with U's Euclidean gradient G given
    (pspec_rhess, the form for the truncated-CG loop of one Newton step): returns (RH, MG, F_col)."""
    ldu = _on_graph(graph, U)
    ldv = _block(V, "V", like=U)
    ldg = _block(G, "G", like=U)
    k = U.shape[1]
    RH = _out_block(RH, "RH", U)
    if MG is None:
        MG = torch.empty((k, k), dtype=torch.float64, device=U.device)
    _fp64_vec(MG, "MG", k * k, U.device)
    F_col = _fcol(F_col, k, U.device)
    ws = _dense_ws(U.device, k)
    _check(lib().pspec_rhess(graph.handle, _dtype_code(U), k, U.data_ptr(), ldu, V.data_ptr(), ldv, G.data_ptr(), ldg,
                             float(p), float(eps), RH.data_ptr(), RH.stride(0), MG.data_ptr(), F_col.data_ptr(),
                             ws.data_ptr(), ws.numel(), _stream(U.device)))
    return RH, MG, F_col


STATIC_K_MAX = 32


def rhvp_static(graph: Graph, U: torch.Tensor, V: torch.Tensor, p: float, eps: float, RH: torch.Tensor,
                RG: torch.Tensor, MG: torch.Tensor, F_col: torch.Tensor):
    """pspec_rhvp_static: rhvp with the library's per-GPU static scratch instead of a workspace, for
    callers that cannot allocate (k <= STATIC_K_MAX).  Every output is the caller's: this wrapper
    allocates nothing.  Calls that overlap on one GPU race (one scratch array per GPU)."""
    ldu = _on_graph(graph, U)
    ldv = _block(V, "V", like=U)
    k = U.shape[1]
    _block(RH, "RH", like=U)
    _block(RG, "RG", like=U)
    _fp64_vec(MG, "MG", k * k, U.device)
    _fp64_vec(F_col, "F_col", k, U.device)
    _check(lib().pspec_rhvp_static(graph.handle, _dtype_code(U), k, U.data_ptr(), ldu, V.data_ptr(), ldv, float(p),
                                   float(eps), RH.data_ptr(), RH.stride(0), RG.data_ptr(), RG.stride(0),
                                   MG.data_ptr(), F_col.data_ptr(), _stream(U.device)))
    return RH, RG, MG, F_col


def project(U: torch.Tensor, Z: torch.Tensor, X: torch.Tensor | None = None, MX: torch.Tensor | None = None,
            out: torch.Tensor | None = None, M: torch.Tensor | None = None):
    """out = Z - U (U^T Z) - X MX; returns (out, M = U^T Z)."""
    ldu = _block(U, "U")
    n, k = U.shape
    ldz = _block(Z, "Z", like=U)
    ldx = _block(X, "X", like=U) if X is not None else 0
    if (X is None) != (MX is None):
        raise PSpecArgError("X and MX go together")
    if MX is not None:
        _fp64_vec(MX, "MX", k * k, U.device)
    out = _out_block(out, "out", U)
    if M is None:
        M = torch.empty((k, k), dtype=torch.float64, device=U.device)
    _fp64_vec(M, "M", k * k, U.device)
    ws = _dense_ws(U.device, k)
    _check(lib().pspec_project(n, k, _dtype_code(U), U.data_ptr(), ldu, Z.data_ptr(), ldz, _ptr(X), ldx, _ptr(MX),
                               out.data_ptr(), out.stride(0), M.data_ptr(), ws.data_ptr(), ws.numel(),
                               _stream(U.device)))
    return out, M


def retract(U: torch.Tensor, eta: torch.Tensor, t: float, out: torch.Tensor | None = None):
    """qf(U + t eta) by Cholesky-QR; returns (Q, R)."""
    ldu = _block(U, "U")
    n, k = U.shape
    lde = _block(eta, "eta", like=U)
    out = _out_block(out, "Uout", U)
    R = torch.empty((k, k), dtype=torch.float64, device=U.device)
    ws = _dense_ws(U.device, k)
    _check(lib().pspec_retract(n, k, _dtype_code(U), U.data_ptr(), ldu, eta.data_ptr(), lde, float(t),
                               out.data_ptr(), out.stride(0), R.data_ptr(), ws.data_ptr(), ws.numel(),
                               _stream(U.device)))
    return out, R


def dot(A: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Frobenius inner product in FP64 (0-dim device tensor)."""
    lda = _block(A, "A")
    n, k = A.shape
    ldb = _block(B, "B", like=A)
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=A.device)
    _fp64_vec(out, "out", 1, A.device)
    ws = _dense_ws(A.device, k)
    _check(lib().pspec_dot(n, k, _dtype_code(A), A.data_ptr(), lda, B.data_ptr(), ldb, out.data_ptr(),
                           ws.data_ptr(), ws.numel(), _stream(A.device)))
    return out


def axpby(alpha: float, X: torch.Tensor, beta: float, Y: torch.Tensor) -> torch.Tensor:
    """Y <- alpha X + beta Y, in place; returns Y."""
    ldy = _block(Y, "Y")
    n, k = Y.shape
    ldx = _block(X, "X", like=Y)
    _check(lib().pspec_axpby(n, k, _dtype_code(Y), float(alpha), X.data_ptr(), ldx, float(beta), Y.data_ptr(),
                             ldy, _stream(Y.device)))
    return Y


KMEANS_MAX = 32


def kmeans_step(X: torch.Tensor, C: torch.Tensor, labels: torch.Tensor | None = None,
                dist: torch.Tensor | None = None, stats: torch.Tensor | None = None, want_labels: bool = True):
    """One Lloyd step on the rows of X (n x d, float32/float64) with FP64 centroids C (c x d):
    returns (labels int32 [n] or None, dist float64 [n] or None, stats float64 [c, d + 2]) where
    stats[j] = (coordinate sums of cluster j, its size, its distance sum).  ``dist`` is written only
    when a tensor is passed."""
    ldx = _block(X, "X")
    n, d = X.shape
    if not (C.is_cuda and C.dtype == torch.float64 and C.dim() == 2 and C.shape[1] == d and C.is_contiguous()
            and C.device == X.device):
        raise PSpecArgError("C must be a contiguous c x d float64 tensor on X's device")
    c = C.shape[0]
    if labels is None and want_labels:
        labels = torch.empty(n, dtype=torch.int32, device=X.device)
    if stats is None:
        stats = torch.empty(c, d + 2, dtype=torch.float64, device=X.device)
    for t, name, dt, size in ((labels, "labels", torch.int32, n), (dist, "dist", torch.float64, n),
                              (stats, "stats", torch.float64, c * (d + 2))):
        if t is not None and (not t.is_cuda or t.dtype != dt or t.numel() != size or not t.is_contiguous()
                              or t.device != X.device):
            raise PSpecArgError(f"{name} must be a contiguous {dt} tensor of {size} elements on X's device")
    nbytes = int(lib().pspec_kmeans_workspace_bytes(c, d))
    key = (str(X.device), _stream(X.device), "kmeans", c, d)
    ws = _ws_cache.get(key)
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
        _ws_cache[key] = ws
    _check(lib().pspec_kmeans_step(n, d, _dtype_code(X), _ptr(X), ldx, c, _ptr(C), _ptr(labels), _ptr(dist),
                                   _ptr(stats), _ptr(ws), nbytes, _stream(X.device)))
    return labels, dist, stats


def rcm_order(rowptr, col) -> np.ndarray:
    """Reverse Cuthill-McKee relabelling of a symmetric host CSR graph: perm[old id] = new id
    (computed by the library on the host; apply it with gen.relabel and to the rows of U)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    n = len(rowptr) - 1
    perm = np.empty(max(n, 0), dtype=np.int64)
    _check(lib().pspec_rcm_order(n, rowptr.ctypes.data, col.ctypes.data, perm.ctypes.data))
    return perm
