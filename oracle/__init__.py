"""FP64 CPU oracle for the p-Laplacian hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this package.
It shares no code with the HIP library: the edge sums are plain C loops in
``pspec_oracle.c`` (IEEE double, libm ``pow``), and the Grassmann steps below are the plain
textbook definitions in NumPy float64.

What each function follows (the paper is Pasadakis, Schenk, Vlacic, Yzelman, "Nonlinear
spectral clustering with C++ GraphBLAS"):

* ``objective``        Eq. (1): F_p(U) = sum_l sum_ij w_ij |u_i - u_j|^p / (2 ||u^l||_p^p),
                       with the p-norm of Section 2.
* ``plap``             the graph p-Laplacian of Section 2, (Delta_p u)_i = sum_j w_ij phi_p(u_i - u_j).
* ``grad``             the EucGrad callback of Section 2: the gradient of Eq. (1), derived by calculus.
* ``hvp``              the EucHessianEta callback of Section 2 / Algorithm 1: the exact Hessian of
                       Eq. (1) applied per column, |x|^(p-2) capped at eps^(p-2) near x = 0.
* ``hvp_sparse``       Algorithm 1 read with sparse matrices D[l], H[l]: the Hessian without its
                       dense rank-2 part, i.e. (p/D) times the derivative of Delta_p u - F phi_p(u).
* ``brute_objective``  Eq. (1) literally: a double loop over all ordered node pairs of a dense W.
* ``project``          Grassmann tangent projection P_U(Z) = Z - U (U^T Z) (Edelman, Arias, Smith
                       geometry cited in Section 1; the paper prints no formula).
* ``riemannian_hessian``  P_U(H eta) - eta (U^T G), the Grassmann Hessian of an extrinsic function.
* ``retract``          qf(U + t eta): the Q factor of the thin QR factorisation with diag(R) > 0.
* ``kmeans_step``      one Lloyd step of the k-means discretisation of the rows of U (Section 1):
                       nearest centroid by squared Euclidean distance (coordinates summed in order,
                       first minimum wins), per-cluster sums, sizes and distance sums.
* ``lloyd``            Lloyd iterations from given centroids until the centroids stop changing.
* ``error_scales``     not a result of the method: per-entry forward-error scales of G and HV (sums
                       of the absolute values of their terms) that the parity tests bound the
                       GPU's differences by.

Every function's pins live in ``tests/test_oracle.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "pspec_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")


def build(src: str = SRC, out: str = LIB, openmp: bool = True) -> str:
    """Compile the C oracle with gcc (no GPU involved)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c99", src, "-o", out, "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.run(cmd, check=True)
    return out


_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_dbl = ctypes.c_double
_i64 = ctypes.c_int64


class Oracle:
    """ctypes front-end of one build of ``pspec_oracle.c``."""

    def __init__(self, path: str | None = None):
        if path is None:
            path = LIB
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
                build()
        self.path = path
        lib = ctypes.CDLL(path)
        opt = ctypes.c_void_p  # nullable double* arguments
        lib.oracle_objective.argtypes = [_i64, _i64p, _i32p, _f64p, ctypes.c_int, _f64p, _i64, _dbl,
                                         opt, opt, opt, opt]
        lib.oracle_objective.restype = None
        lib.oracle_plap.argtypes = [_i64, _i64p, _i32p, _f64p, ctypes.c_int, _f64p, _i64, _dbl, _f64p]
        lib.oracle_plap.restype = None
        lib.oracle_grad.argtypes = [_i64, _i64p, _i32p, _f64p, ctypes.c_int, _f64p, _i64, _dbl, _f64p, opt]
        lib.oracle_grad.restype = None
        lib.oracle_hvp.argtypes = [_i64, _i64p, _i32p, _f64p, ctypes.c_int, _f64p, _i64, _f64p, _i64,
                                   _dbl, _dbl, _f64p, opt, opt]
        lib.oracle_hvp.restype = None
        lib.oracle_hvp_sparse.argtypes = [_i64, _i64p, _i32p, _f64p, ctypes.c_int, _f64p, _i64, _f64p, _i64,
                                          _dbl, _dbl, _f64p]
        lib.oracle_hvp_sparse.restype = None
        lib.oracle_error_scales.argtypes = [_i64, _i64p, _i32p, _f64p, ctypes.c_int, _f64p, _i64, _f64p, _i64,
                                            _dbl, _dbl, _f64p, _f64p, opt]
        lib.oracle_error_scales.restype = None
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_num_threads.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        self.lib = lib

    @staticmethod
    def _csr(rowptr, col, w):
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        w = np.ascontiguousarray(w, dtype=np.float64)
        if rowptr.ndim != 1 or len(rowptr) < 2 or rowptr[0] != 0 or len(col) != rowptr[-1] or len(w) != len(col):
            raise ValueError("malformed CSR")
        return rowptr, col, w

    @staticmethod
    def _block(A, n):
        A = np.ascontiguousarray(A, dtype=np.float64)
        if A.ndim != 2 or A.shape[0] != n:
            raise ValueError("block must be n x k")
        return A

    def num_threads(self) -> int:
        return int(self.lib.oracle_num_threads())

    def set_num_threads(self, t: int) -> None:
        """Threads of the later calls (the OpenMP row loops); sums over rows stay sequential."""
        self.lib.oracle_set_num_threads(int(t))

    def objective(self, rowptr, col, w, U, p):
        """Returns (F, Fcol, Ncol, Dcol) of Eq. (1)."""
        rowptr, col, w = self._csr(rowptr, col, w)
        n = len(rowptr) - 1
        U = self._block(U, n)
        k = U.shape[1]
        N = np.zeros(k)
        D = np.zeros(k)
        Fc = np.zeros(k)
        F = np.zeros(1)
        self.lib.oracle_objective(n, rowptr, col, w, k, U, k, float(p), N.ctypes.data, D.ctypes.data,
                                  Fc.ctypes.data, F.ctypes.data)
        return float(F[0]), Fc, N, D

    def plap(self, rowptr, col, w, U, p):
        """Returns Delta_p applied to every column of U (n x k)."""
        rowptr, col, w = self._csr(rowptr, col, w)
        n = len(rowptr) - 1
        U = self._block(U, n)
        L = np.zeros_like(U)
        self.lib.oracle_plap(n, rowptr, col, w, U.shape[1], U, U.shape[1], float(p), L)
        return L

    def grad(self, rowptr, col, w, U, p):
        """Returns (G, Fcol): the Euclidean gradient of Eq. (1) and the per-column objective."""
        rowptr, col, w = self._csr(rowptr, col, w)
        n = len(rowptr) - 1
        U = self._block(U, n)
        k = U.shape[1]
        G = np.zeros_like(U)
        Fc = np.zeros(k)
        self.lib.oracle_grad(n, rowptr, col, w, k, U, k, float(p), G, Fc.ctypes.data)
        return G, Fc

    def hvp(self, rowptr, col, w, U, V, p, eps):
        """Returns (HV, G, Fcol): the Hessian of Eq. (1) at U applied to V, the gradient, F per column."""
        rowptr, col, w = self._csr(rowptr, col, w)
        n = len(rowptr) - 1
        U = self._block(U, n)
        V = self._block(V, n)
        k = U.shape[1]
        if V.shape[1] != k:
            raise ValueError("U and V differ in k")
        HV = np.zeros_like(U)
        G = np.zeros_like(U)
        Fc = np.zeros(k)
        self.lib.oracle_hvp(n, rowptr, col, w, k, U, k, V, k, float(p), float(eps), HV, G.ctypes.data,
                            Fc.ctypes.data)
        return HV, G, Fc

    def hvp_sparse(self, rowptr, col, w, U, V, p, eps):
        """The sparse part of the Hessian at U applied to V: the derivative of (p/D)(Delta_p u - F phi_p(u))
        along V with D and F held fixed (the exact Hessian without its rank-2 term)."""
        rowptr, col, w = self._csr(rowptr, col, w)
        n = len(rowptr) - 1
        U = self._block(U, n)
        V = self._block(V, n)
        k = U.shape[1]
        if V.shape[1] != k:
            raise ValueError("U and V differ in k")
        HV = np.zeros_like(U)
        self.lib.oracle_hvp_sparse(n, rowptr, col, w, k, U, k, V, k, float(p), float(eps), HV)
        return HV


    def error_scales(self, rowptr, col, w, U, V, p, eps, sparse=False):
        """Returns (SG, SH): per-entry forward-error scales of the gradient and of the Hessian-vector
        product (absolute-value sums of their terms, each power term weighted by its conditioning;
        see oracle_error_scales); with ``sparse`` also SHs, the scale of the Hessian's sparse part.
        For parity tolerances |x_gpu - x| <= tau * S, not a result of the method."""
        rowptr, col, w = self._csr(rowptr, col, w)
        n = len(rowptr) - 1
        U = self._block(U, n)
        V = self._block(V, n)
        k = U.shape[1]
        if V.shape[1] != k:
            raise ValueError("U and V differ in k")
        SG = np.zeros_like(U)
        SH = np.zeros_like(U)
        SHs = np.zeros_like(U) if sparse else None
        self.lib.oracle_error_scales(n, rowptr, col, w, k, U, k, V, k, float(p), float(eps), SG, SH,
                                     None if SHs is None else SHs.ctypes.data)
        return (SG, SH, SHs) if sparse else (SG, SH)


_default: Oracle | None = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def brute_objective(W, U, p) -> float:
    """Eq. (1) written literally over a dense weight matrix: all ordered pairs (i, j).

    Pure Python loops; meant for n of a few dozen at most.
    """
    W = np.asarray(W, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    n, k = U.shape
    total = 0.0
    for l in range(k):
        num = 0.0
        for i in range(n):
            for j in range(n):
                num += W[i, j] * abs(U[i, l] - U[j, l]) ** p
        den = 0.0
        for i in range(n):
            den += abs(U[i, l]) ** p
        total += num / (2.0 * den)
    return total


def project(U, Z):
    """P_U(Z) = Z - U (U^T Z) for U with orthonormal columns; also returns M = U^T Z."""
    U = np.asarray(U, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    M = U.T @ Z
    return Z - U @ M, M


def riemannian_hessian(U, G, HV, eta):
    """P_U(H eta) - eta (U^T G): Riemannian Hessian on Gr(k, n) from Euclidean G and H eta."""
    U = np.asarray(U, dtype=np.float64)
    P, _ = project(U, HV)
    return P - np.asarray(eta, dtype=np.float64) @ (U.T @ np.asarray(G, dtype=np.float64))


def retract(U, eta, t):
    """qf(U + t eta): Q of the thin QR factorisation with a positive diagonal of R."""
    Y = np.asarray(U, dtype=np.float64) + t * np.asarray(eta, dtype=np.float64)
    Q, R = np.linalg.qr(Y, mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def kmeans_step(X, C):
    """Assign every row of X to its nearest centroid (rows of C) and gather the cluster statistics.

    dist[i, j] = sum_t (X[i, t] - C[j, t])^2, accumulated over t in order with each square rounded
    before it is added; labels = first index of the row minimum.  Returns (labels int32, dist of the
    chosen centroid, stats) with stats[j] = [sum of the member rows, member count, sum of their dist].
    """
    X = np.asarray(X, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    n, d = X.shape
    c = C.shape[0]
    D = np.zeros((n, c))
    for t in range(d):
        D = D + (X[:, t:t + 1] - C[None, :, t]) ** 2
    labels = np.argmin(D, axis=1) if n else np.zeros(0, dtype=np.int64)
    dist = D[np.arange(n), labels]
    stats = np.zeros((c, d + 2))
    for j in range(c):
        m = labels == j
        stats[j, :d] = X[m].sum(axis=0)
        stats[j, d] = m.sum()
        stats[j, d + 1] = dist[m].sum()
    return labels.astype(np.int32), dist, stats


def lloyd(X, C0, iters=100):
    """Lloyd's k-means from the centroids C0: assign, move every non-empty cluster's centroid to its
    mean (an empty cluster keeps its centroid), stop when the centroids no longer change.  Returns
    (labels, centroids, inertia, steps) with labels and inertia taken against the final centroids."""
    C = np.array(C0, dtype=np.float64)
    d = C.shape[1]
    for step in range(1, iters + 1):
        labels, dist, stats = kmeans_step(X, C)
        cnt = stats[:, d]
        Cn = C.copy()
        nz = cnt > 0
        Cn[nz] = stats[nz, :d] / cnt[nz, None]
        if np.array_equal(Cn, C):
            return labels, C, float(dist.sum()), step
        C = Cn
    labels, dist, _ = kmeans_step(X, C)
    return labels, C, float(dist.sum()), iters
