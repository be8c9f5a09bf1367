"""Host driver: Riemannian Newton with truncated CG on Gr(k, n), p-continuation, k-means, RCut.

Section 2 of the paper minimises Eq. (1) "for progressively smaller values of p" with Newton's
method on the Grassmann manifold, each Newton system solved by truncated conjugate gradients,
then discretises the eigenvectors with k-means; Section 3.1 scores the clusters with
RCut = sum_i cut(C_i, complement) / |C_i|.  The paper gives no schedule or tolerances; the choices
below are this implementation's (see the readings in the design notes):

* geometry: P_U(Z) = Z - U U^T Z, Riemannian gradient P_U(G), Riemannian Hessian
  P_U(H eta) - eta (U^T G), retraction qf(U + t eta) (all on the GPU through the C ABI);
* Newton: Steihaug-Toint truncated CG (stop on negative curvature, or when
  ||r|| <= ||g|| min(||g||^theta, kappa)) inside a trust region whose radius follows the ratio of
  actual to model decrease (`rtr`, the default), or followed by Armijo backtracking on
  F(R_U(t eta)) (`Solver.newton`);
* p-continuation: p = 2.0, 1.8, ... down to the target, each level warm-started;
* k-means: Lloyd iterations on the GPU (one pspec_kmeans_step pass per iteration) from k-means++
  seeds (fixed seed, several restarts) on the rows of U.

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

    def __init__(self, graph: pspec.Graph, k: int, dtype=torch.float32, eps: float = 1e-8,
                 hessian: str = "exact"):
        """``hessian``: "exact" (the Hessian of Eq. (1)) or "sparse" (without its rank-2 part: Algorithm 1
        read with sparse D[l], H[l]; Newton then solves an approximate system)."""
        if hessian not in ("exact", "sparse"):
            raise ValueError(f"unknown hessian {hessian!r}")
        self.graph, self.k, self.dtype, self.eps, self.hessian = graph, k, dtype, eps, hessian
        n = graph.n
        dev = graph.device
        mk = lambda: torch.empty((n, k), dtype=dtype, device=dev)  # noqa: E731
        self.G, self.HV, self.rgrad = mk(), mk(), mk()
        self.eta, self.r, self.delta, self.Hd, self.Ut = mk(), mk(), mk(), mk(), mk()
        self.MG = torch.empty((k, k), dtype=torch.float64, device=dev)
        self.Hd2 = mk() if hessian == "sparse" else None

    # --- small wrappers (each a library call) -------------------------------------------------
    def F(self, U, p) -> float:
        F, _ = pspec.objective(self.graph, U, p)
        return float(F.item())

    def dot(self, A, B) -> float:
        return float(pspec.dot(A, B).item())

    def hess(self, U, p, X, out, G=None):
        """Riemannian Hessian at U applied to the tangent vector X.  With G, the Euclidean gradient at
        U (computed once per Newton step, as the truncated-CG loops below do), one pspec_rhess call
        (edge pass without the gradient rows, epilogue, Gram matrices, projection); without it, G is
        formed first."""
        if self.hessian == "exact":
            if G is None:
                pspec.grad(self.graph, U, p, G=self.G)
                G = self.G
            pspec.rhess(self.graph, U, X, G, p, self.eps, RH=out, MG=self.MG)
            return out
        # sparse-only operator: Euclidean product, then P_U(H X) - X (U^T G)
        pspec.hvp(self.graph, U, X, p, self.eps, HV=self.HV, G=self.G, sparse_only=True)
        pspec.project(U, self.G, out=self.Hd2, M=self.MG)
        pspec.project(U, self.HV, X=X, MX=self.MG, out=out)
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
                self.hess(U, p, self.delta, self.Hd, G=self.G)
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


@dataclass
class TrustRegionOptions:
    max_outer: int = 60
    rel_tol: float = 1e-5       # stop when ||grad|| <= rel_tol * ||grad at the first iterate||
    abs_tol: float = 0.0
    tcg_max: int = 60
    kappa: float = 0.1
    theta: float = 1.0
    rho_accept: float = 0.1     # accept the step when the actual/model decrease ratio exceeds this
    delta_bar: float | None = None  # largest radius (default sqrt(k))
    delta0: float | None = None     # first radius (default delta_bar / 8)


def rtr(solver: Solver, U: torch.Tensor, p: float, opt: TrustRegionOptions | None = None, progress=None):
    """Riemannian trust-region Newton on Gr(k, n) (Absil, Baker and Gallivan's RTR, the method behind
    the paper's Newton / truncated-CG solver): the Newton system is solved by Steihaug-Toint
    truncated CG inside a ball of radius Delta, the step is accepted by the ratio rho of actual to
    model decrease, and Delta shrinks or grows with rho.  ``progress(it, F, |grad|, tCG steps)`` is
    called after every outer iteration when given.  Returns the final U and a log."""
    opt = opt or TrustRegionOptions()
    s = solver
    k = s.k
    delta_bar = opt.delta_bar if opt.delta_bar is not None else float(k) ** 0.5
    delta = opt.delta0 if opt.delta0 is not None else delta_bar / 8.0
    info = NewtonInfo(p=p)
    U = pspec.axpby(1.0, U, 0.0, torch.empty_like(U))  # working copy
    Heta = torch.empty_like(U)
    g0 = None
    Fu = s.F(U, p)  # kept from the accepted trial point afterwards: every F here is one objective call
    for it in range(opt.max_outer):
        pspec.grad(s.graph, U, p, G=s.G)
        pspec.project(U, s.G, out=s.rgrad, M=s.MG)
        gg = s.dot(s.rgrad, s.rgrad)
        gn = gg ** 0.5
        info.F.append(Fu)
        info.grad_norm.append(gn)
        if g0 is None:
            g0 = gn
        if gn <= max(opt.abs_tol, opt.rel_tol * g0) or not np.isfinite(gn):
            break
        # Steihaug-Toint truncated CG for Hess[eta] = -grad within ||eta|| <= delta
        pspec.axpby(0.0, s.rgrad, 0.0, s.eta)
        pspec.axpby(0.0, s.rgrad, 0.0, Heta)
        pspec.axpby(1.0, s.rgrad, 0.0, s.r)
        pspec.axpby(-1.0, s.r, 0.0, s.delta)
        rr, r0 = gg, gn
        e_e, e_d, d_d = 0.0, 0.0, gg  # <eta,eta>, <eta,delta>, <delta,delta> by recurrence
        nt = 0
        for j in range(opt.tcg_max):
            nt = j + 1
            s.hess(U, p, s.delta, s.Hd, G=s.G)
            dHd = s.dot(s.delta, s.Hd)
            alpha = rr / dHd if dHd > 0.0 else 0.0
            e_e_new = e_e + 2.0 * alpha * e_d + alpha * alpha * d_d
            if dHd <= 0.0 or e_e_new >= delta * delta:
                # to the boundary along delta: ||eta + tau delta|| = delta, tau >= 0
                tau = (-e_d + ((e_d * e_d + d_d * (delta * delta - e_e)) ** 0.5)) / d_d
                pspec.axpby(tau, s.delta, 1.0, s.eta)
                pspec.axpby(tau, s.Hd, 1.0, Heta)
                break
            e_e = e_e_new
            pspec.axpby(alpha, s.delta, 1.0, s.eta)
            pspec.axpby(alpha, s.Hd, 1.0, Heta)
            pspec.axpby(alpha, s.Hd, 1.0, s.r)
            rr_new = s.dot(s.r, s.r)
            if rr_new ** 0.5 <= r0 * min(r0 ** opt.theta, opt.kappa):
                break
            beta = rr_new / rr
            rr = rr_new
            e_d = beta * (e_d + alpha * d_d)
            d_d = rr + beta * beta * d_d
            pspec.axpby(-1.0, s.r, beta, s.delta)
        info.tcg_iterations.append(nt)
        # model decrease m(0) - m(eta) = -<grad, eta> - 1/2 <eta, Hess eta>
        model = -s.dot(s.rgrad, s.eta) - 0.5 * s.dot(s.eta, Heta)
        eta_norm = s.dot(s.eta, s.eta) ** 0.5
        pspec.retract(U, s.eta, 1.0, out=s.Ut)
        Ft = s.F(s.Ut, p)
        rho = (Fu - Ft) / model if model > 0.0 else -1.0
        if rho < 0.25:
            delta *= 0.25
        elif rho > 0.75 and eta_norm >= 0.99 * delta:
            delta = min(2.0 * delta, delta_bar)
        F_it = Fu
        if rho > opt.rho_accept:
            pspec.axpby(1.0, s.Ut, 0.0, U)
            Fu = Ft
        info.iterations = it + 1
        if progress is not None:
            progress(it + 1, F_it, gn, nt)
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


def lloyd_gpu(X: torch.Tensor, C0: np.ndarray, iters: int = 100):
    """Lloyd's k-means on the rows of the device block X from the centroids C0 (c x d): every step is
    one pspec.kmeans_step pass over X; the new centroids (cluster means; an empty cluster keeps its
    centroid) are formed on the host from the c x (d + 2) statistics.  Stops when the centroids no
    longer change.  Returns (labels: device int32, centroids: host float64, inertia, steps), labels
    and inertia taken against the returned centroids."""
    C = np.array(C0, dtype=np.float64)
    c, d = C.shape
    labels = torch.empty(X.shape[0], dtype=torch.int32, device=X.device)
    stats = torch.empty(c, d + 2, dtype=torch.float64, device=X.device)
    Cd = torch.empty(c, d, dtype=torch.float64, device=X.device)
    for step in range(1, iters + 1):
        Cd.copy_(torch.from_numpy(C))
        pspec.kmeans_step(X, Cd, labels=labels, stats=stats)
        st = stats.cpu().numpy()
        cnt = st[:, d]
        Cn = C.copy()
        nz = cnt > 0
        Cn[nz] = st[nz, :d] / cnt[nz, None]
        if np.array_equal(Cn, C):
            return labels, C, float(st[:, d + 1].sum()), step
        C = Cn
    Cd.copy_(torch.from_numpy(C))
    pspec.kmeans_step(X, Cd, labels=labels, stats=stats)
    return labels, C, float(stats[:, d + 1].sum().item()), iters


def kmeans_gpu(X: torch.Tensor, k: int, seed: int = 0, n_init: int = 3, iters: int = 100):
    """k-means of the rows of the device block X into k clusters: k-means++ seeds (each new seed drawn
    with probability proportional to the squared distance to the nearest seed so far, the distances
    from pspec.kmeans_step), then Lloyd iterations on the GPU; of n_init restarts the one with the
    lowest inertia wins.  Returns (labels: host int64, centroids, inertia)."""
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    dist = torch.empty(n, dtype=torch.float64, device=X.device)
    best = None
    for _ in range(n_init):
        idx = [int(rng.integers(n))]
        for _c in range(1, k):
            seeds = X[idx].double().contiguous()
            pspec.kmeans_step(X, seeds, dist=dist, want_labels=False)
            d2 = dist.cpu().numpy()
            tot = d2.sum()
            idx.append(int(rng.choice(n, p=d2 / tot)) if tot > 0 else int(rng.integers(n)))
        labels, C, inertia, _ = lloyd_gpu(X, X[idx].double().cpu().numpy(), iters)
        if best is None or inertia < best[2]:
            best = (labels.cpu().numpy().astype(np.int64), C, inertia)
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
            seed: int = 0, opt=None, step: float = 0.2, method: str = "rtr"):
    """p-spectral clustering: continuation from p = 2 to p, a Riemannian Newton solve at each level
    (method "rtr": trust region, TrustRegionOptions; "newton": Armijo line search, NewtonOptions),
    then k-means on the rows of U.

    Returns (labels, U, infos, rcut_value); host_graph supplies the CSR used by RCut.
    """
    if method not in ("rtr", "newton"):
        raise ValueError(f"unknown method {method!r}")
    solver = Solver(graph, k, dtype, eps)
    U = orthonormal_start(graph.n, k, seed, dtype, graph.device)
    infos = []
    for pl in p_levels(p, step):
        if method == "rtr":
            U, info = rtr(solver, U, pl, opt)
        else:
            U, info = solver.newton(U, pl, opt)
        infos.append(info)
    labels, _, _ = kmeans_gpu(U, k, seed=seed)
    return labels, U, infos, rcut(host_graph.rowptr, host_graph.col, host_graph.w, labels)


def delaunay_study(r: int, k: int = 4, p: float = 1.2, step: float = 0.2, dtype=torch.float64,
                   seed: int = 0, opt: TrustRegionOptions | None = None, save: str | None = None,
                   log=print, spec_opt: TrustRegionOptions | None = None, order: str = "rcm",
                   resume: str | None = None, time_rhvp: bool = True) -> dict:
    """The whole pipeline on a Delaunay graph of 2^r uniform random points (the stand-in for the
    paper's triangulation matrices, Section 3): trust-region Newton at each p level of the
    continuation, k-means on the rows of U and RCut after every level.  The p = 2 level is the
    spectral (Spec) solution the smaller-p levels are compared with; ``spec_opt`` (default ``opt``)
    sets its limits, since the p = 2 Newton system of a planar graph grows ill-conditioned with n
    and needs more CG steps than the levels after it.  ``order`` "rcm" relabels the graph by the
    library's reverse Cuthill-McKee order before the solve (the points are numbered at random, so
    without it every neighbour gather misses the caches); "points" keeps the point order.  The
    Riemannian HVP call is timed once per graph (``rhvp_ms``, p = 1.5) unless ``time_rhvp`` is off.
    With ``save`` set, U is written to ``save/U_r{r}_p{p:.2f}.npy`` after each level; with ``resume``
    set to such a directory, the last level saved there is loaded (and clustered again) and the
    continuation goes on from the next level; every kernel is deterministic, so a resumed run ends
    with the same U as an uninterrupted one.  Returns a dict with one entry per level."""
    import os
    import time

    from . import gen

    if order not in ("rcm", "points"):
        raise ValueError(f"unknown order {order!r}")
    t0 = time.perf_counter()
    g = gen.delaunay(1 << r, seed=seed)
    t_graph = time.perf_counter() - t0
    t_order = 0.0
    if order == "rcm":
        t0 = time.perf_counter()
        g = gen.relabel(g, pspec.rcm_order(g.rowptr, g.col), "rcm")
        t_order = time.perf_counter() - t0
    dg = pspec.Graph.from_host(g, "cuda", k_max=k)
    solver = Solver(dg, k, dtype, 1e-8)
    U = orthonormal_start(g.n, k, seed, dtype, "cuda")
    out = {"r": r, "n": g.n, "edges": g.nnz // 2, "k": k, "dtype": str(dtype).replace("torch.", ""),
           "order": order, "graph_seconds": round(t_graph, 2), "order_seconds": round(t_order, 2),
           "rhvp_ms": _time_rhvp(dg, U, 1.5) if time_rhvp else None, "levels": []}
    if time_rhvp:
        log(f"r={r} n={g.n} order={order} rhvp {out['rhvp_ms']:.3f} ms")
    checkpoint = lambda d, pl: os.path.join(d, f"U_r{r}_p{pl:.2f}.npy")  # noqa: E731
    levels = p_levels(p, step)
    start = 0
    if resume:
        saved = [i for i, pl in enumerate(levels) if os.path.exists(checkpoint(resume, pl))]
        if saved:
            i = saved[-1]
            U = torch.as_tensor(np.load(checkpoint(resume, levels[i]))).to(dtype).to("cuda").contiguous()
            labels, _, _ = kmeans_gpu(U, k, seed=seed)
            out["levels"].append({"p": levels[i], "resumed": True, "F": solver.F(U, levels[i]),
                                  "rcut": rcut(g.rowptr, g.col, g.w, labels)})
            log(f"r={r} resumed after p={levels[i]:.2f} from {resume}")
            start = i + 1
    for pl in levels[start:]:
        t1 = time.perf_counter()
        def every10(it, F, gn, nt, pl=pl):
            if it % 10 == 0:
                log(f"r={r} p={pl:.2f}   outer {it:3d} F {F:.6e} |g| {gn:.2e} tcg {nt}")

        U, info = rtr(solver, U, pl, spec_opt if (pl == 2.0 and spec_opt is not None) else opt, every10)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t1
        Uh = U.double().cpu().numpy()
        labels, _, _ = kmeans_gpu(U, k, seed=seed)
        lev = {"p": pl, "outer": info.iterations, "tcg": int(sum(info.tcg_iterations)), "F": info.F[-1],
               "grad_rel": info.grad_norm[-1] / info.grad_norm[0], "rcut": rcut(g.rowptr, g.col, g.w, labels),
               "solve_seconds": round(t_solve, 2)}
        out["levels"].append(lev)
        log(f"r={r} p={pl:.2f} outer {lev['outer']:3d} tcg {lev['tcg']:5d} F {lev['F']:.6e} "
            f"|g|/|g0| {lev['grad_rel']:.1e} RCut {lev['rcut']:.5f} {t_solve:.1f}s")
        if save:
            os.makedirs(save, exist_ok=True)
            np.save(checkpoint(save, pl), Uh)
    spec, last = out["levels"][0]["rcut"], out["levels"][-1]["rcut"]
    out["rcut_spec"], out["rcut_pspec"] = spec, last
    out["rcut_gain_percent"] = 100.0 * (spec - last) / spec
    return out


def _time_rhvp(dg: pspec.Graph, U: torch.Tensor, p: float, reps: int = 20) -> float:
    """Milliseconds per Riemannian HVP call (pspec_rhvp) at U along V = U."""
    RH, RG = torch.empty_like(U), torch.empty_like(U)
    pspec.rhvp(dg, U, U, p, 1e-8, RH=RH, RG=RG)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        pspec.rhvp(dg, U, U, p, 1e-8, RH=RH, RG=RG)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def main(argv=None):
    import argparse
    import json

    ap = argparse.ArgumentParser(description="p-spectral clustering of Delaunay graphs of 2^r random points "
                                             "in the unit square: RCut at p = 2 against the smallest p")
    ap.add_argument("--r", type=int, nargs="+", default=[16])
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--p", type=float, default=1.2)
    ap.add_argument("--step", type=float, default=0.2)
    ap.add_argument("--dtype", choices=["f32", "f64"], default="f64")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-outer", type=int, default=60)
    ap.add_argument("--tcg-max", type=int, default=60)
    ap.add_argument("--rel-tol", type=float, default=None)
    ap.add_argument("--spec-max-outer", type=int, default=100, help="outer limit at p = 2")
    ap.add_argument("--spec-tcg-max", type=int, default=300, help="tCG limit at p = 2")
    ap.add_argument("--save", default=None, help="directory for U after each p level (.npy)")
    ap.add_argument("--resume", default=None, help="continue after the last level saved in this directory")
    ap.add_argument("--order", choices=["rcm", "points"], default="rcm",
                    help="node numbering: reverse Cuthill-McKee (default) or the random point order")
    a = ap.parse_args(argv)
    dtype = torch.float64 if a.dtype == "f64" else torch.float32
    rel = a.rel_tol if a.rel_tol is not None else (1e-6 if dtype == torch.float64 else 1e-4)
    opt = TrustRegionOptions(max_outer=a.max_outer, tcg_max=a.tcg_max, rel_tol=rel)
    spec = TrustRegionOptions(max_outer=a.spec_max_outer, tcg_max=a.spec_tcg_max, rel_tol=rel)
    for r in a.r:
        res = delaunay_study(r, a.k, a.p, a.step, dtype, a.seed, opt, a.save,
                             log=lambda s: print(s, flush=True), spec_opt=spec, order=a.order, resume=a.resume)
        print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
