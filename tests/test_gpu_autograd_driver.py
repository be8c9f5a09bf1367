"""GPU: the torch.autograd.Function wrappers (checked against central finite differences and the
FP64 oracle gradient) and the Newton-tCG clustering driver."""
import numpy as np
import pytest
import torch

from paper_2605_26975_amd import autograd as pag
from paper_2605_26975_amd import driver, gen, pspec
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def grid128():
    """The 3-D 6-neighbour 128^3 grid (2,097,152 nodes), k = 8, p = 1.2."""
    return gen.grid3d(128)


def _away_from_kinks(g, U, V, delta=1e-2):
    """V with zeros wherever a central difference along V could cross a kink of |x|^(p-1) or
    |u|^(p-1): at both ends of every edge with |u_i - u_j| < delta and where |u_i| < delta, per
    column.  Along h V every edge difference and entry then stays at least delta - 2 h max|V| from
    its kink (h <= 1e-4, max|V| ~ 6: at least 8.8e-3, eight times the step).
    Returns the masked V and the number of zeroed entries."""
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    near = np.abs(U[rows] - U[g.col]) < delta
    zero = np.abs(U) < delta
    np.logical_or.at(zero, rows, near)
    Vm = np.where(zero, 0.0, V).astype(V.dtype)
    return Vm, int(zero.sum())


def test_autograd_gradient_vs_oracle_and_fd(grid128):
    g = grid128
    k, p, eps = 8, 1.2, 1e-8
    print(f"[case] grid128 autograd k={k} p={p}", flush=True)
    U, V = gu.inputs(g.n, k)
    dg = gu.device_graph(g, k)
    # FP32 autograd gradient against the FP64 oracle gradient
    U32 = torch.as_tensor(U).cuda().requires_grad_(True)
    F32 = pag.objective(U32, dg, p, eps)
    (G32,) = torch.autograd.grad(F32, U32)
    _, Go, Fco = gu.oracle_hvp(g, U, V, p, eps)
    SG, _ = gu.oracle_scales(g, U, V, p, eps)
    G32h = G32.double().cpu().numpy()
    assert gu.rel(G32h, Go) < 1e-5 and gu.colmax(G32h, Go) < 1e-5
    assert gu.ew(G32h, Go, SG) <= gu.TOLS[torch.float32]["tau"]
    assert abs(float(F32.detach()) - Fco.sum()) / Fco.sum() < 1e-5
    # FP64 path: directional derivative against a central difference of F.  F (~36) is a sum of
    # 12.5M terms whose FP64 rounding noise, ~1e-13 of F, the difference divides by 2 hF: at
    # hF = 1e-4 that is ~2e-8 against a derivative of ~7e-4, and the O(hF^2) truncation (every
    # difference stays >= 8.8e-3 from a kink) is smaller still; at 1e-6 the noise alone would be
    # ~3e-5 of the derivative.
    hF = 1e-4
    Vm, zeroed = _away_from_kinks(g, U, V)
    print(f"direction zeroed at {zeroed} of {V.size} entries near kinks")
    assert zeroed < 0.05 * V.size
    U64 = torch.as_tensor(U).double().cuda().requires_grad_(True)
    V64 = torch.as_tensor(Vm).double().cuda()
    F64 = pag.objective(U64, dg, p, eps)
    (G64,) = torch.autograd.grad(F64, U64, create_graph=True)
    with torch.no_grad():
        Fp = float(pag.objective(U64 + hF * V64, dg, p, eps))
        Fm = float(pag.objective(U64 - hF * V64, dg, p, eps))
    fd = (Fp - Fm) / (2 * hF)
    an = float((G64 * V64).sum())
    assert abs(an - fd) <= 1e-4 * abs(fd), (an, fd)


def test_autograd_hvp_vs_fd_and_forward_mode(grid128):
    g = grid128
    k, p, eps, h = 8, 1.2, 1e-8, 1e-6
    print(f"[case] grid128 hvp fd k={k} p={p}", flush=True)
    U, V = gu.inputs(g.n, k)
    dg = gu.device_graph(g, k)
    Vm, zeroed = _away_from_kinks(g, U, V)
    print(f"direction zeroed at {zeroed} of {V.size} entries near kinks")
    U64 = torch.as_tensor(U).double().cuda().requires_grad_(True)
    V64 = torch.as_tensor(Vm).double().cuda()
    # reverse-over-reverse: d/dU <G(U), V> = H V
    F = pag.objective(U64, dg, p, eps)
    (G,) = torch.autograd.grad(F, U64, create_graph=True)
    (HV_rr,) = torch.autograd.grad(G, U64, grad_outputs=V64)
    # forward-over-reverse: forward-mode derivative of the gradient along V
    import torch.autograd.forward_ad as fwAD

    with fwAD.dual_level():
        G_dual = pag.gradient(fwAD.make_dual(U64.detach(), V64), dg, p, eps)
        HV_fr = fwAD.unpack_dual(G_dual).tangent
    assert torch.equal(HV_rr, HV_fr)
    # central difference of the gradient, row by row away from the kinks of |x|^(p-1)
    with torch.no_grad():
        Gp = pag.gradient(U64 + h * V64, dg, p, eps)
        Gm = pag.gradient(U64 - h * V64, dg, p, eps)
    fd = ((Gp - Gm) / (2 * h)).cpu().numpy()
    hv = HV_rr.cpu().numpy()
    err = np.linalg.norm(hv - fd) / np.linalg.norm(fd)
    print(f"HVP vs central difference of the gradient: {err:.2e}")
    assert err < 1e-5, err
    # the FP32 HVP kernel against the FP64 oracle on the same inputs
    HVo, Go, Fco = gu.oracle_hvp(g, U, V, p, eps)
    SG, SH = gu.oracle_scales(g, U, V, p, eps)
    HV32, G32, Fc32 = gu.gpu_hvp(dg, U, V, p, eps, torch.float32)
    gu.check(gu.errors(HV32, G32, Fc32, HVo, Go, Fco, SG, SH), torch.float32)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_cluster_sbm1000_recovers_blocks(dtype):
    g = gen.sbm_bernoulli(1000, 4, 0.05, 0.002)
    truth = np.repeat(np.arange(4), 250)
    dg = gu.device_graph(g, 4)
    for p in (2.0, 1.3):
        print(f"[case] cluster sbm1000 {dtype} p={p}", flush=True)
        labels, U, infos, rc = driver.cluster(dg, g, 4, p, dtype=dtype)
        acc = driver.matched_accuracy(labels, truth)
        print(f"p={p} accuracy={acc:.4f} RCut={rc:.5f} newton={[i.iterations for i in infos]}")
        assert acc >= 0.95
        Uh = U.double().cpu().numpy()
        assert np.max(np.abs(Uh.T @ Uh - np.eye(4))) < (1e-5 if dtype == torch.float32 else 1e-12)


def test_cluster_knn_fp32_matches_fp64():
    """kNN mixture (100k points, k = 8, p = 1.3): FP32 and FP64 labels agree.  With
    w = exp(-d^2 / s^2) and s ~ 0.056 many tail points have weights that round to 0 in FP32, so the
    minimiser isolates them (RCut ~ 2e-4) and labels do not follow the mixture components; the
    comparison is FP32 against FP64."""
    g = gen.knn_mixture(100_000, 8, 10, 1.0, 20.0)
    truth = g.meta["labels"]
    dg = gu.device_graph(g, 8)
    out = {}
    for dtype in (torch.float32, torch.float64):
        print(f"[case] cluster knn100k {dtype}", flush=True)
        labels, U, infos, rc = driver.cluster(dg, g, 8, 1.3, dtype=dtype)
        out[dtype] = labels
        print(f"{dtype}: accuracy vs mixture {driver.matched_accuracy(labels, truth):.4f} RCut {rc:.5f}")
    agree = driver.matched_accuracy(out[torch.float32], out[torch.float64])
    print(f"FP32 vs FP64 label agreement {agree:.5f}")
    assert agree >= 0.99


def _laplacian_eigs(g, k):
    """The k smallest eigenvalues of L = D - W, by a dense symmetric eigensolve (small graphs)."""
    W = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    W[rows, g.col] = g.w
    L = np.diag(W.sum(axis=1)) - W
    return np.linalg.eigvalsh(L)[:k]


def test_rtr_p2_reaches_the_laplacian_eigenvalue_sum():
    """At p = 2 and orthonormal U, F_2(U) = tr(U^T L U) (N sums over ordered pairs), whose minimum on
    Gr(k, n) is the sum of the k smallest eigenvalues of L (Ky Fan).  The trust-region Newton from a
    random start must reach it, never go below it, and never increase F."""
    n, k = 2048, 4
    g = gen.delaunay(n, seed=3)
    print(f"[case] rtr delaunay n={n} k={k} p=2", flush=True)
    lam = _laplacian_eigs(g, k)
    dg = gu.device_graph(g, k)
    solver = driver.Solver(dg, k, torch.float64, 1e-8)
    U0 = driver.orthonormal_start(n, k, 0, torch.float64, "cuda")
    opt = driver.TrustRegionOptions(max_outer=300, rel_tol=1e-10, tcg_max=300)
    U, info = driver.rtr(solver, U0, 2.0, opt)
    F = np.asarray(info.F)
    print(f"outer {info.iterations} tcg {sum(info.tcg_iterations)} F {F[-1]:.12f} sum(lambda) {lam.sum():.12f}")
    assert info.grad_norm[-1] <= 1e-10 * info.grad_norm[0]
    assert np.all(np.diff(F) <= 1e-13 * F[:-1])
    assert F[-1] >= lam.sum() * (1.0 - 1e-12)
    assert abs(F[-1] - lam.sum()) <= 1e-8 * lam.sum() + 1e-12
    # the minimiser spans the eigenspace: U stays orthonormal and L U = U (U^T L U)
    Uh = U.cpu().numpy()
    assert np.abs(Uh.T @ Uh - np.eye(k)).max() < 1e-12


def test_rtr_continuation_decreases_f_at_each_level():
    """From the p = 2 minimiser, each smaller p level only accepts steps that lower F_p."""
    n, k = 4096, 4
    g = gen.delaunay(n, seed=4)
    print(f"[case] rtr continuation delaunay n={n} k={k}", flush=True)
    dg = gu.device_graph(g, k)
    for dtype in (torch.float32, torch.float64):
        solver = driver.Solver(dg, k, dtype, 1e-8)
        U = driver.orthonormal_start(n, k, 0, dtype, "cuda")
        for pl in (2.0, 1.8, 1.6):
            U, info = driver.rtr(solver, U, pl, driver.TrustRegionOptions(max_outer=25, rel_tol=1e-6))
            F = np.asarray(info.F)
            tol = 1e-6 if dtype == torch.float32 else 1e-13
            print(f"{dtype} p={pl} outer {info.iterations} F {F[0]:.6f} -> {F[-1]:.6f}")
            assert np.all(np.diff(F) <= tol * F[:-1])
            assert F[-1] < F[0]


def test_sparse_hessian_equals_exact_on_tangents_at_p2_only():
    """At p = 2, phi(u) = u and tangent vectors X satisfy U^T X = 0, so the rank-2 part of the
    Hessian, -(p/D)(g phi^T + phi g^T) X, lies in span(U) after a = phi^T x = 0 and is removed by
    P_U: the Riemannian Hessians of the exact and sparse-only operators coincide.  Below p = 2 they
    differ; the trust-region Newton with the sparse model still only accepts descent steps."""
    n, k = 4096, 4
    g = gen.delaunay(n, seed=7)
    print(f"[case] sparse hessian delaunay n={n} k={k}", flush=True)
    dg = gu.device_graph(g, k)
    ex = driver.Solver(dg, k, torch.float64, 1e-8)
    sp = driver.Solver(dg, k, torch.float64, 1e-8, hessian="sparse")
    U = driver.orthonormal_start(n, k, 0, torch.float64, "cuda")
    X, _ = pspec.project(U, torch.as_tensor(gen.block(n, k, gen.SEED_V)).double().cuda())
    for p, same in ((2.0, True), (1.6, False)):
        He = ex.hess(U, p, X, torch.empty_like(X)).cpu().numpy()
        Hs = sp.hess(U, p, X, torch.empty_like(X)).cpu().numpy()
        d = gu.rel(Hs, He)
        print(f"p={p} rel diff {d:.2e}")
        assert (d < 1e-10) if same else (d > 1e-6)
    U2, _ = driver.rtr(ex, U, 2.0, driver.TrustRegionOptions(max_outer=20, rel_tol=1e-6))
    _, info = driver.rtr(sp, U2, 1.6, driver.TrustRegionOptions(max_outer=20, rel_tol=1e-6))
    F = np.asarray(info.F)
    assert np.all(np.diff(F) <= 1e-13 * F[:-1]) and F[-1] < F[0]


def test_delaunay_study_resumes_to_the_same_solution(tmp_path):
    """A run stopped after p = 2 and resumed from its checkpoint ends with the same U, bit for bit,
    as the uninterrupted run (every kernel and host step is deterministic)."""
    import os

    print("[case] delaunay study resume r=11", flush=True)
    opt = driver.TrustRegionOptions(max_outer=15, rel_tol=1e-8)
    full, part = str(tmp_path / "full"), str(tmp_path / "part")
    a = driver.delaunay_study(11, k=4, p=1.6, step=0.2, opt=opt, save=full, log=print, time_rhvp=False)
    os.makedirs(part)
    name = "U_r11_p2.00.npy"
    with open(os.path.join(full, name), "rb") as f, open(os.path.join(part, name), "wb") as g:
        g.write(f.read())
    b = driver.delaunay_study(11, k=4, p=1.6, step=0.2, opt=opt, save=part, resume=part, log=print,
                              time_rhvp=False)
    assert b["levels"][0].get("resumed") and [lv["p"] for lv in b["levels"]] == [2.0, 1.8, 1.6]
    assert np.array_equal(np.load(os.path.join(full, "U_r11_p1.60.npy")),
                          np.load(os.path.join(part, "U_r11_p1.60.npy")))
    assert b["rcut_pspec"] == a["rcut_pspec"]


@pytest.mark.parametrize("p", [2.0, 1.3])
def test_fp32_parity_at_a_driver_iterate(p):
    """Near a stationary point the gradient G = (p/D)(L - F phi_p(u)) is a difference of nearly
    equal terms (at p = 2 exactly L u - lambda u), so its FP32 error relative to |G| grows while
    its error relative to the terms it is made of does not.  At the trust-region iterate of SBM-1000
    (FP64 solve, continuation to p) every entry of the FP32 G and HV stays within tau of its
    forward-error scale; the block errors relative to ||G||, ||HV|| and to ||L|| are printed."""
    g = gen.sbm_bernoulli(1000, 4, 0.05, 0.002)
    k, eps = 4, 1e-8
    print(f"[case] parity at driver iterate sbm1000 p={p}", flush=True)
    dg = gu.device_graph(g, k)
    solver = driver.Solver(dg, k, torch.float64, eps)
    U = driver.orthonormal_start(g.n, k, 0, torch.float64, "cuda")
    for pl in driver.p_levels(p):
        U, info = driver.rtr(solver, U, pl, driver.TrustRegionOptions(max_outer=60, rel_tol=1e-8))
    print(f"p={p}: |grad_R| {info.grad_norm[0]:.3e} -> {info.grad_norm[-1]:.3e}")
    # the iterate and a tangent direction, rounded to FP32 once (both sides see the same values)
    U32 = U.float().cpu().numpy()
    V0 = gen.block(g.n, k, gen.SEED_V).astype(np.float64)
    Uh = U32.astype(np.float64)
    V32 = (V0 - Uh @ (Uh.T @ V0)).astype(np.float32)
    e = gu.compare(g, k, p, eps, torch.float32, U=U32, V=V32, dg=dg)
    L = orc_plap(g, U32, p)
    HVo, Go, _ = gu.oracle_hvp(g, U32, V32, p, eps)
    HV32, G32, _ = gu.gpu_hvp(dg, U32, V32, p, eps, torch.float32)
    scale = (p / np.sum(np.abs(Uh) ** p, axis=0))
    print(f"|G|/|p L/D| = {np.linalg.norm(Go) / np.linalg.norm(scale * L):.2e};  FP32 G error rel |G| {e['G']:.2e}, "
          f"rel |p L/D| {np.linalg.norm(G32 - Go) / np.linalg.norm(scale * L):.2e};  HV rel {e['HV']:.2e}")
    gu.check(e, torch.float32, norms=False)
    # the Riemannian gradient P_U(G), which does vanish at the stationary point, and the Riemannian
    # Hessian: element-wise against their forward-error scales, relative errors printed
    import oracle as orc

    Ut = torch.as_tensor(U32).cuda()
    Vt = torch.as_tensor(V32).cuda()
    RH, RG, _, _ = pspec.rhvp(dg, Ut, Vt, p, eps)
    RGo, _ = orc.project(Uh, Go)
    RHo = orc.riemannian_hessian(Uh, Go, HVo, V32.astype(np.float64))
    SG, SH = gu.oracle_scales(g, U32, V32, p, eps)
    aU, aV = np.abs(Uh), np.abs(V32.astype(np.float64))
    RGh, RHh = RG.double().cpu().numpy(), RH.double().cpu().numpy()
    wRG = gu.ew(RGh, RGo, SG + aU @ (aU.T @ SG))
    wRH = gu.ew(RHh, RHo, SH + aU @ (aU.T @ SH) + aV @ (aU.T @ SG))
    print(f"|P_U G| / |G| = {np.linalg.norm(RGo) / np.linalg.norm(Go):.2e}; FP32 P_U G error rel |P_U G| "
          f"{gu.rel(RGh, RGo):.2e}, element-wise {wRG:.2e}; Riemannian HV rel {gu.rel(RHh, RHo):.2e}, "
          f"element-wise {wRH:.2e}")
    assert wRG <= gu.TOLS[torch.float32]["tau"] and wRH <= gu.TOLS[torch.float32]["tau"]


def orc_plap(g, U, p):
    import oracle as orc

    return orc.default().plap(g.rowptr, g.col, g.w.astype(np.float64), U.astype(np.float64), p)
