"""Host driver: Riemannian Newton with truncated CG on Gr(k, n), p-continuation, k-means, RCut.

Section 2 of the paper minimises Eq. (1) "for progressively smaller values of p" with Newton's
method on the Grassmann manifold, each Newton system solved by truncated conjugate gradients,
then discretises the eigenvectors with k-means; Section 3.1 scores the clusters with
RCut = sum_i cut(C_i, complement) / |C_i|.  The paper gives no schedule or tolerances; the choices
below are this implementation's (see the readings in the design notes):

* geometry: P_U(Z) = Z - U U^T Z, Riemannian gradient P_U(G), Riemannian Hessian
  P_U(H eta) - eta (U^T G), retraction qf(U + t eta) (all on the GPU through the C ABI);
* Newton: Steihaug-Toint truncated CG (stop on negative curvature, or when
  ||r|| <= ||g|| min(||g||^theta, kappa)), then Armijo backtracking on F(R_U(t eta));
* p-continuation: p = 2.0, 1.8, ... down to the target, each level warm-started;
* k-means: Lloyd iterations from k-means++ seeds (fixed seed, several restarts) on the rows of U.

Every vector operation (inner products, axpby, projections, retractions, the objective,
gradient and Hessian-vector products) runs in the HIP library; only FP64 scalars cross to the
host, a few per truncated-CG iteration.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import pspec


@dataclass
class NewtonOptions:
    max_newton: int = 25
    rel_tol: float = 1e-5  # stop when ||grad|| <= rel_tol * ||grad at the first iterate||
    abs_tol: float = 0.0
    tcg_max: int = 40
    kappa: float = 0.1
    theta: float = 1.0
    armijo: float = 1e-4
    max_backtracks: int = 30


@dataclass
class NewtonInfo:
    p: float
    iterations: int = 0
    tcg_iterations: list = field(default_factory=list)
    F: list = field(default_factory=list)
    grad_norm: list = field(default_factory=list)


class Solver:
    """Work buffers and the Newton-tCG iteration for one graph, k and dtype."""

    def __init__(self, graph: pspec.Graph, k: int, dtype=torch.float32, eps: float = 1e-8):
        self.graph, self.k, self.dtype, self.eps = graph, k, dtype, eps
        n = graph.n
        dev = graph.device
        mk = lambda: torch.empty((n, k), dtype=dtype, device=dev)  # noqa: E731
        self.G, self.HV, self.rgrad = mk(), mk(), mk()
        self.eta, self.r, self.delta, self.Hd, self.Ut = mk(), mk(), mk(), mk(), mk()
        self.MG = torch.empty((k, k), dtype=torch.float64, device=dev)

    # --- small wrappers (each a library call) -------------------------------------------------
    def F(self, U, p) -> float:
        F, _ = pspec.objective(self.graph, U, p)
        return float(F.item())

    def dot(self, A, B) -> float:
        return float(pspec.dot(A, B).item())

    def hess(self, U, p, X, out):
        """Riemannian Hessian at U applied to the tangent vector X: one fused library call (edge
        pass, epilogue, both Gram matrices and the projection); the Riemannian gradient it also
        returns goes to a scratch block."""
        pspec.rhvp(self.graph, U, X, p, self.eps, RH=out, RG=self.HV, MG=self.MG)
        return out

    def newton(self, U: torch.Tensor, p: float, opt: NewtonOptions | None = None) -> tuple[torch.Tensor, NewtonInfo]:
        """Minimise F_p over Gr(k, n) from U (orthonormal columns); returns the final U and a log."""
        opt = opt or NewtonOptions()
        info = NewtonInfo(p=p)
        U = pspec.axpby(1.0, U, 0.0, torch.empty_like(U))  # working copy
        g0 = None
        for it in range(opt.max_newton):
            pspec.grad(self.graph, U, p, G=self.G)
            pspec.project(U, self.G, out=self.rgrad, M=self.MG)
            gn = self.dot(self.rgrad, self.rgrad) ** 0.5
            Fu = self.F(U, p)
            info.F.append(Fu)
            info.grad_norm.append(gn)
            if g0 is None:
                g0 = gn
            if gn <= max(opt.abs_tol, opt.rel_tol * g0) or not np.isfinite(gn):
                break
            # truncated CG on the tangent space: Hess[eta] = -grad
            pspec.axpby(0.0, self.rgrad, 0.0, self.eta)
            pspec.axpby(1.0, self.rgrad, 0.0, self.r)
            pspec.axpby(-1.0, self.r, 0.0, self.delta)
            rr = gn * gn
            r0 = gn
            nt = 0
            for j in range(opt.tcg_max):
                nt = j + 1
                self.hess(U, p, self.delta, self.Hd)
                dHd = self.dot(self.delta, self.Hd)
                if dHd <= 0.0:
                    if j == 0:
                        pspec.axpby(1.0, self.delta, 0.0, self.eta)  # steepest descent
                    break
                alpha = rr / dHd
                pspec.axpby(alpha, self.delta, 1.0, self.eta)
                pspec.axpby(alpha, self.Hd, 1.0, self.r)
                rr_new = self.dot(self.r, self.r)
                if rr_new ** 0.5 <= r0 * min(r0 ** opt.theta, opt.kappa):
                    break
                beta = rr_new / rr
                rr = rr_new
                pspec.axpby(-1.0, self.r, beta, self.delta)
            info.tcg_iterations.append(nt)
            slope = self.dot(self.rgrad, self.eta)
            if not slope < 0.0:  # not a descent direction: fall back to -grad
                pspec.axpby(-1.0, self.rgrad, 0.0, self.eta)
                slope = -gn * gn
            t = 1.0
            accepted = False
            for _ in range(opt.max_backtracks):
                pspec.retract(U, self.eta, t, out=self.Ut)
                if self.F(self.Ut, p) <= Fu + opt.armijo * t * slope:
                    accepted = True
                    break
                t *= 0.5
            if not accepted:
                break
            pspec.axpby(1.0, self.Ut, 0.0, U)
            info.iterations = it + 1
        return U, info


def orthonormal_start(n: int, k: int, seed: int, dtype=torch.float32, device="cuda") -> torch.Tensor:
    """qf(X) of a seeded N(0, 1) block (retraction with t = 0)."""
    from . import gen

    X = torch.as_tensor(gen.block(n, k, seed)).to(dtype).to(device)
    Q, _ = pspec.retract(X, X, 0.0)
    return Q


def p_levels(p_target: float, step: float = 0.2) -> list[float]:
    levels = [2.0]
    p = 2.0
    while p - step > p_target + 1e-12:
        p = round(p - step, 10)
        levels.append(p)
    if levels[-1] != p_target:
        levels.append(p_target)
    return levels


def kmeans(X: np.ndarray, k: int, seed: int = 0, n_init: int = 5, iters: int = 100) -> np.ndarray:
    """Lloyd's k-means from k-means++ seeds; the restart with the lowest inertia wins."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    best, best_inertia = None, np.inf
    for _ in range(n_init):
        C = np.empty((k, X.shape[1]))
        C[0] = X[rng.integers(n)]
        d2 = np.sum((X - C[0]) ** 2, axis=1)
        for c in range(1, k):
            prob = d2 / d2.sum() if d2.sum() > 0 else np.full(n, 1.0 / n)
            C[c] = X[rng.choice(n, p=prob)]
            d2 = np.minimum(d2, np.sum((X - C[c]) ** 2, axis=1))
        labels = np.zeros(n, dtype=np.int64)
        for _it in range(iters):
            dist = np.sum(X * X, axis=1)[:, None] - 2.0 * X @ C.T + np.sum(C * C, axis=1)[None, :]
            new = np.argmin(dist, axis=1)
            if _it > 0 and np.array_equal(new, labels):
                break
            labels = new
            for c in range(k):
                m = labels == c
                if np.any(m):
                    C[c] = X[m].mean(axis=0)
        inertia = float(np.sum((X - C[labels]) ** 2))
        if inertia < best_inertia:
            best, best_inertia = labels.copy(), inertia
    return best


def rcut(rowptr: np.ndarray, col: np.ndarray, w: np.ndarray, labels: np.ndarray) -> float:
    """RCut = sum_c cut(C_c, complement) / |C_c| (Section 3.1), from a symmetric CSR."""
    labels = np.asarray(labels)
    n = len(labels)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    cross = labels[rows] != labels[col]
    k = int(labels.max()) + 1
    cut = np.bincount(labels[rows[cross]], weights=np.asarray(w, dtype=np.float64)[cross], minlength=k)
    size = np.bincount(labels, minlength=k)
    return float(np.sum(cut[size > 0] / size[size > 0]))


def matched_accuracy(a: np.ndarray, b: np.ndarray) -> float:
    """Fraction of nodes whose labels agree after the best one-to-one relabelling (Hungarian)."""
    from scipy.optimize import linear_sum_assignment

    ka, kb = int(a.max()) + 1, int(b.max()) + 1
    M = np.zeros((ka, kb))
    np.add.at(M, (a, b), 1)
    r, c = linear_sum_assignment(-M)
    return float(M[r, c].sum() / len(a))


def cluster(graph: pspec.Graph, host_graph, k: int, p: float, dtype=torch.float32, eps: float = 1e-8,
            seed: int = 0, opt: NewtonOptions | None = None, step: float = 0.2):
    """p-spectral clustering: continuation from p = 2 to p, Newton-tCG at each level, then k-means.

    Returns (labels, U, infos, rcut_value); host_graph supplies the CSR used by RCut.
    """
    solver = Solver(graph, k, dtype, eps)
    U = orthonormal_start(graph.n, k, seed, dtype, graph.device)
    infos = []
    for pl in p_levels(p, step):
        U, info = solver.newton(U, pl, opt)
        infos.append(info)
    labels = kmeans(U.double().cpu().numpy(), k, seed=seed)
    return labels, U, infos, rcut(host_graph.rowptr, host_graph.col, host_graph.w, labels)
