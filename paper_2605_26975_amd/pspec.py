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
        "pspec_graph_create": [i64, i64, vp, vp, vp, i32, i32, vp, ctypes.POINTER(vp)],
        "pspec_graph_destroy": [vp],
        "pspec_graph_info": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "pspec_graph_set_timing_events": [vp, vp, vp],
        "pspec_objective": [vp, i32, i32, vp, i64, dbl, vp, vp, vp],
        "pspec_grad": [vp, i32, i32, vp, i64, dbl, vp, i64, vp, vp],
        "pspec_hvp": [vp, i32, i32, vp, i64, vp, i64, dbl, dbl, vp, i64, vp, i64, vp, vp],
        "pspec_hvp_sparse": [vp, i32, i32, vp, i64, vp, i64, dbl, dbl, vp, i64, vp, i64, vp, vp],
        "pspec_rhvp": [vp, i32, i32, vp, i64, vp, i64, dbl, dbl, vp, i64, vp, i64, vp, vp, vp, sz, vp],
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
        "pspec_graph_create", "pspec_graph_destroy", "pspec_graph_info", "pspec_graph_set_timing_events",
        "pspec_objective", "pspec_grad",
        "pspec_hvp", "pspec_hvp_sparse", "pspec_rhvp", "pspec_dense_workspace_bytes", "pspec_project", "pspec_retract", "pspec_dot",
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
    raise TypeError(f"unsupported dtype {t.dtype}")


def _block(t: torch.Tensor, name: str) -> int:
    """Validate an n x k row-major device block; return its leading dimension."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be 2-D with unit column stride (row-major)")
    return t.stride(0)


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
    """A device CSR graph with its row schedule (pspec_graph_create).  Keeps the CSR tensors alive."""

    def __init__(self, rowptr: torch.Tensor, col: torch.Tensor, w: torch.Tensor, k_max: int):
        for t, name, dt in ((rowptr, "rowptr", torch.int64), (col, "col", torch.int32)):
            if not t.is_cuda or t.dtype != dt or t.dim() != 1 or not t.is_contiguous():
                raise TypeError(f"{name} must be a contiguous 1-D {dt} device tensor")
        if not w.is_cuda or w.dim() != 1 or not w.is_contiguous():
            raise TypeError("w must be a contiguous 1-D device tensor")
        self.rowptr, self.col, self.w = rowptr, col, w
        self.n = rowptr.numel() - 1
        self.nnz = col.numel()
        self.k_max = k_max
        self.device = rowptr.device
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().pspec_graph_create(self.n, self.nnz, rowptr.data_ptr(), col.data_ptr(), w.data_ptr(),
                                            _dtype_code(w), k_max, _stream(self.device), ctypes.byref(self._h)))

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
        return dict(heavy_rows=h.value, chunks=c.value, split_rows=s.value)

    def set_timing_events_raw(self, before, after) -> None:
        """Record two raw hipEvent_t handles (or None, None) around the edge pass of later calls."""
        _check(lib().pspec_graph_set_timing_events(self.handle, before, after))

    def close(self) -> None:
        if self._h:
            _check(lib().pspec_graph_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def objective(graph: Graph, U: torch.Tensor, p: float, F_col: torch.Tensor | None = None,
              F: torch.Tensor | None = None):
    """Eq. (1): returns (F, F_col) as FP64 device tensors (0-dim and k)."""
    ldu = _block(U, "U")
    k = U.shape[1]
    if F_col is None:
        F_col = torch.empty(k, dtype=torch.float64, device=U.device)
    if F is None:
        F = torch.empty((), dtype=torch.float64, device=U.device)
    _check(lib().pspec_objective(graph.handle, _dtype_code(U), k, U.data_ptr(), ldu, float(p), F_col.data_ptr(),
                                 F.data_ptr(), _stream(U.device)))
    return F, F_col


def grad(graph: Graph, U: torch.Tensor, p: float, G: torch.Tensor | None = None, F_col: torch.Tensor | None = None):
    """Euclidean gradient of Eq. (1): returns (G, F_col)."""
    ldu = _block(U, "U")
    k = U.shape[1]
    if G is None:
        G = torch.empty_like(U, memory_format=torch.contiguous_format)
    if F_col is None:
        F_col = torch.empty(k, dtype=torch.float64, device=U.device)
    _check(lib().pspec_grad(graph.handle, _dtype_code(U), k, U.data_ptr(), ldu, float(p), G.data_ptr(),
                            _block(G, "G"), F_col.data_ptr(), _stream(U.device)))
    return G, F_col


def hvp(graph: Graph, U: torch.Tensor, V: torch.Tensor, p: float, eps: float = 1e-8,
        HV: torch.Tensor | None = None, G: torch.Tensor | None = None, F_col: torch.Tensor | None = None,
        sparse_only: bool = False):
    """Hessian of Eq. (1) at U applied to V, fused with the gradient: returns (HV, G, F_col).
    ``sparse_only`` drops the dense rank-2 part of the Hessian (pspec_hvp_sparse)."""
    ldu, ldv = _block(U, "U"), _block(V, "V")
    k = U.shape[1]
    if HV is None:
        HV = torch.empty(U.shape, dtype=U.dtype, device=U.device)
    if G is None:
        G = torch.empty(U.shape, dtype=U.dtype, device=U.device)
    if F_col is None:
        F_col = torch.empty(k, dtype=torch.float64, device=U.device)
    fn = lib().pspec_hvp_sparse if sparse_only else lib().pspec_hvp
    _check(fn(graph.handle, _dtype_code(U), k, U.data_ptr(), ldu, V.data_ptr(), ldv, float(p), float(eps),
              HV.data_ptr(), _block(HV, "HV"), G.data_ptr(), _block(G, "G"), F_col.data_ptr(), _stream(U.device)))
    return HV, G, F_col


def rhvp(graph: Graph, U: torch.Tensor, V: torch.Tensor, p: float, eps: float = 1e-8,
         RH: torch.Tensor | None = None, RG: torch.Tensor | None = None, MG: torch.Tensor | None = None,
         F_col: torch.Tensor | None = None):
    """Riemannian Hessian at U applied to the tangent vector V and Riemannian gradient, fused:
    returns (RH = P_U(H V) - V (U^T G), RG = P_U(G), MG = U^T G, F_col)."""
    ldu, ldv = _block(U, "U"), _block(V, "V")
    k = U.shape[1]
    if RH is None:
        RH = torch.empty(U.shape, dtype=U.dtype, device=U.device)
    if RG is None:
        RG = torch.empty(U.shape, dtype=U.dtype, device=U.device)
    if MG is None:
        MG = torch.empty((k, k), dtype=torch.float64, device=U.device)
    if F_col is None:
        F_col = torch.empty(k, dtype=torch.float64, device=U.device)
    ws = _dense_ws(U.device, k)
    _check(lib().pspec_rhvp(graph.handle, _dtype_code(U), k, U.data_ptr(), ldu, V.data_ptr(), ldv, float(p),
                            float(eps), RH.data_ptr(), _block(RH, "RH"), RG.data_ptr(), _block(RG, "RG"),
                            MG.data_ptr(), F_col.data_ptr(), ws.data_ptr(), ws.numel(), _stream(U.device)))
    return RH, RG, MG, F_col


def project(U: torch.Tensor, Z: torch.Tensor, X: torch.Tensor | None = None, MX: torch.Tensor | None = None,
            out: torch.Tensor | None = None, M: torch.Tensor | None = None):
    """out = Z - U (U^T Z) - X MX; returns (out, M = U^T Z)."""
    n, k = U.shape
    if out is None:
        out = torch.empty(U.shape, dtype=U.dtype, device=U.device)
    if M is None:
        M = torch.empty((k, k), dtype=torch.float64, device=U.device)
    ws = _dense_ws(U.device, k)
    _check(lib().pspec_project(n, k, _dtype_code(U), U.data_ptr(), _block(U, "U"), Z.data_ptr(), _block(Z, "Z"),
                               _ptr(X), _block(X, "X") if X is not None else 0, _ptr(MX), out.data_ptr(),
                               _block(out, "out"), M.data_ptr(), ws.data_ptr(), ws.numel(), _stream(U.device)))
    return out, M


def retract(U: torch.Tensor, eta: torch.Tensor, t: float, out: torch.Tensor | None = None):
    """qf(U + t eta) by Cholesky-QR; returns (Q, R)."""
    n, k = U.shape
    if out is None:
        out = torch.empty(U.shape, dtype=U.dtype, device=U.device)
    R = torch.empty((k, k), dtype=torch.float64, device=U.device)
    ws = _dense_ws(U.device, k)
    _check(lib().pspec_retract(n, k, _dtype_code(U), U.data_ptr(), _block(U, "U"), eta.data_ptr(),
                               _block(eta, "eta"), float(t), out.data_ptr(), _block(out, "Uout"), R.data_ptr(),
                               ws.data_ptr(), ws.numel(), _stream(U.device)))
    return out, R


def dot(A: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Frobenius inner product in FP64 (0-dim device tensor)."""
    n, k = A.shape
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=A.device)
    ws = _dense_ws(A.device, k)
    _check(lib().pspec_dot(n, k, _dtype_code(A), A.data_ptr(), _block(A, "A"), B.data_ptr(), _block(B, "B"),
                           out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(A.device)))
    return out


def axpby(alpha: float, X: torch.Tensor, beta: float, Y: torch.Tensor) -> torch.Tensor:
    """Y <- alpha X + beta Y, in place; returns Y."""
    n, k = Y.shape
    _check(lib().pspec_axpby(n, k, _dtype_code(Y), float(alpha), X.data_ptr(), _block(X, "X"), float(beta),
                             Y.data_ptr(), _block(Y, "Y"), _stream(Y.device)))
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
    if not (C.is_cuda and C.dtype == torch.float64 and C.dim() == 2 and C.shape[1] == d and C.is_contiguous()):
        raise ValueError("C must be a contiguous c x d float64 device tensor")
    c = C.shape[0]
    if labels is None and want_labels:
        labels = torch.empty(n, dtype=torch.int32, device=X.device)
    if stats is None:
        stats = torch.empty(c, d + 2, dtype=torch.float64, device=X.device)
    for t, name, dt, size in ((labels, "labels", torch.int32, n), (dist, "dist", torch.float64, n),
                              (stats, "stats", torch.float64, c * (d + 2))):
        if t is not None and (not t.is_cuda or t.dtype != dt or t.numel() != size or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {dt} device tensor of {size} elements")
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
