"""GPU: the fused Riemannian gradient and Hessian-vector product (pspec_rhvp) against the unfused
sequence pspec_hvp -> pspec_project(G) -> pspec_project(HV, X = V, MX = U^T G) -- bit for bit, or
entry by entry within the forward-error bound where the Gram products are formed in the edge pass
(FP32, k = 16) -- and against the FP64 oracle's Grassmann formulas (tangent projection and
Riemannian Hessian)."""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_2605_26975_amd import gen, pspec
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _tangent_pair(n, k, seed):
    """U with orthonormal columns and V = P_U(V0) tangent at U, both FP64."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, k)))
    V0 = rng.standard_normal((n, k))
    return U, V0 - U @ (U.T @ V0)


def _place(U, V, dtype, layout):
    k = U.shape[1]
    if layout == "interleaved":
        P = torch.empty((U.shape[0], 2 * k), dtype=dtype, device="cuda")
        P[:, :k] = torch.as_tensor(U).to(dtype)
        P[:, k:] = torch.as_tensor(V).to(dtype)
        return P[:, :k], P[:, k:]
    return torch.as_tensor(U).to(dtype).cuda(), torch.as_tensor(V).to(dtype).cuda()


def _unfused(dg, U, V, p, eps):
    HV, G, Fc = pspec.hvp(dg, U, V, p, eps)
    RG, MG = pspec.project(U, G)
    RH, _ = pspec.project(U, HV, X=V, MX=MG)
    return RH, RG, MG, Fc


_GRAPHS = {
    "sbm20k": lambda: gen.sbm_edges(20_000, 8, 100_000, 12_000, 0.5, 1.5, seed=11),
    "sbm1000": lambda: gen.sbm_bernoulli(1000, 4, 0.05, 0.002),
    # light, single-chunk heavy and split rows (the Gram products of heavy rows come from their own kernel)
    "rmat14": lambda: gen.rmat(14, 16, 0.57, 0.19, 0.19, 0.1, 1.0, seed=9),
}


@pytest.mark.parametrize("layout", ["separate", "interleaved"])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("k", [3, 5, 12, 16, 32, 64])
@pytest.mark.parametrize("graph", ["sbm20k", "sbm1000", "rmat14"])
def test_rhvp_bit_identical_to_hvp_and_projections(graph, k, dtype, layout):
    """Covers the 16-byte and element paths (k a multiple of 4 or not), the register-fused kernels
    (rows of at most 128 bytes) and the stand-alone fallback (FP32 k = 64, FP64 k >= 32), and
    fewer rows than Gram workgroups (n = 1000)."""
    print(f"[case] rhvp bitwise {graph} k={k} {dtype} {layout}", flush=True)
    g = _GRAPHS[graph]()
    Uh, Vh = _tangent_pair(g.n, k, seed=k)
    dg = gu.device_graph(g, k)
    U, V = _place(Uh, Vh, dtype, layout)
    p, eps = 1.3, 1e-8
    got = pspec.rhvp(dg, U, V, p, eps)
    ref = _unfused(dg, U, V, p, eps)
    if not gu.gram_in_edge_pass(k, dtype):
        for name, a, b in zip(("RH", "RG", "MG", "F_col"), got, ref):
            assert torch.equal(a, b), name
        return
    # Gram products formed in the edge pass: equal to rounding, each side within tau of the exact
    # value, so within 2 tau of each other entry by entry
    assert torch.equal(got[3], ref[3])
    Ur, Vr = U.double().cpu().numpy(), V.double().cpu().numpy()
    SG, SH = gu.oracle_scales(g, Ur, Vr, p, eps)
    S_RG, S_RH, S_MG = gu.riemannian_scales(Ur, Vr, SG, SH)
    tau = gu.TOLS[dtype]["tau"]
    for name, a, b, S in zip(("RH", "RG", "MG"), got, ref, (S_RH, S_RG, S_MG)):
        d = gu.ew(a.double().cpu().numpy(), b.double().cpu().numpy(), S)
        print(f"{name} vs unfused, element-wise {d:.2e}", flush=True)
        assert d <= 2 * tau, name


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("k", [8, 16])
@pytest.mark.parametrize("graph", ["sbm30k", "rmat14"])
def test_rhvp_vs_oracle(graph, k, dtype):
    """k = 16 in FP32 forms the Gram products in the edge pass (rmat14: heavy and split rows too)."""
    g = (gen.sbm_edges(30_000, 8, 150_000, 20_000, 0.5, 1.5, seed=12) if graph == "sbm30k"
         else _GRAPHS["rmat14"]())
    p, eps = 1.2, 1e-8
    print(f"[case] rhvp oracle {graph} k={k} {dtype}", flush=True)
    Uh, Vh = _tangent_pair(g.n, k, seed=3)
    U, V = _place(Uh, Vh, dtype, "interleaved")
    # the oracle sees exactly the rounded inputs
    Ur, Vr = U.double().cpu().numpy(), V.double().cpu().numpy()
    dg = gu.device_graph(g, k)
    RH, RG, MG, Fc = pspec.rhvp(dg, U, V, p, eps)
    HVo, Go, Fco = gu.oracle_hvp(g, Ur, Vr, p, eps)
    RGo, MGo = orc.project(Ur, Go)
    RHo = orc.riemannian_hessian(Ur, Go, HVo, Vr)
    # element-wise scales: G's and HV's errors carried through the projections,
    # RG = G - U (U^T G), RH = HV - U (U^T HV) - V (U^T G)
    SG, SH = gu.oracle_scales(g, Ur, Vr, p, eps)
    aU, aV = np.abs(Ur), np.abs(Vr)
    S_RG = SG + aU @ (aU.T @ SG)
    S_RH = SH + aU @ (aU.T @ SH) + aV @ (aU.T @ SG)
    t = gu.TOLS[dtype]
    RGh, RHh = RG.double().cpu().numpy(), RH.double().cpu().numpy()
    e = dict(F=float(np.max(np.abs(Fc.cpu().numpy() - Fco) / np.abs(Fco))),
             MG=gu.ew(MG.cpu().numpy(), MGo, aU.T @ SG), RG=gu.rel(RGh, RGo), RH=gu.rel(RHh, RHo),
             RG_colmax=gu.colmax(RGh, RGo), RH_colmax=gu.colmax(RHh, RHo),
             RG_ew=gu.ew(RGh, RGo, S_RG), RH_ew=gu.ew(RHh, RHo, S_RH))
    print(e)
    assert e["F"] <= t["F"] and e["MG"] <= t["tau"], e
    assert max(e["RG"], e["RH"], e["RG_colmax"], e["RH_colmax"]) <= t["norm"], e
    assert e["RG_ew"] <= t["tau"] and e["RH_ew"] <= t["tau"], e
    # RG is tangent at U, and so is RH (for tangent V the correction term keeps it there)
    Ut = torch.as_tensor(Ur).cuda()
    assert float((Ut.T @ RG.double()).abs().max()) < (1e-5 if dtype == torch.float32 else 1e-12)


def test_rhvp_rejects_bad_arguments():
    g = gen.sbm_bernoulli(1000, 4, 0.05, 0.002)
    dg = gu.device_graph(g, 4)
    U = torch.randn(g.n, 4, device="cuda")
    V = torch.randn(g.n, 4, device="cuda")
    with pytest.raises(pspec.PSpecError):
        pspec.rhvp(dg, U, V, 1.5, 1e-8, RH=U)  # output overlaps U
    with pytest.raises(pspec.PSpecError):
        pspec.rhvp(dg, U, V, 1.5, 0.0)  # eps must be positive
    R = torch.empty_like(U)
    with pytest.raises(pspec.PSpecError):
        pspec.rhvp(dg, U, V, 1.5, 1e-8, RH=R, RG=R)  # outputs overlap each other


@pytest.mark.parametrize("layout", ["separate", "interleaved"])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("k", [3, 5, 12, 16, 32, 64])
def test_rhess_at_fixed_u_matches_rhvp_and_oracle(k, dtype, layout):
    """pspec_rhess (U fixed, its gradient G given, no gradient rows or RG formed): F_col equals
    pspec_rhvp's bit for bit, MG too unless the Gram products are formed in the edge pass (then within
    2 tau of it entry by entry); RH agrees with pspec_rhvp's and with the oracle's Riemannian Hessian
    entry by entry within tau times its forward-error scale (G's and HV's scales carried through the
    projection), on the fused (16 <= k <= 32) and stand-alone paths."""
    print(f"[case] rhess k={k} {dtype} {layout}", flush=True)
    g = _GRAPHS["sbm20k"]()
    Uh, Vh = _tangent_pair(g.n, k, seed=k)
    dg = gu.device_graph(g, k)
    U, V = _place(Uh, Vh, dtype, layout)
    p, eps = 1.3, 1e-8
    RH, RG, MG, Fc = pspec.rhvp(dg, U, V, p, eps)
    G, _ = pspec.grad(dg, U, p)
    RH2, MG2, Fc2 = pspec.rhess(dg, U, V, G, p, eps)
    torch.cuda.synchronize()
    assert torch.equal(Fc, Fc2)
    Ur, Vr = U.double().cpu().numpy(), V.double().cpu().numpy()
    HVo, Go, _ = gu.oracle_hvp(g, Ur, Vr, p, eps)
    RHo = orc.riemannian_hessian(Ur, Go, HVo, Vr)
    SG, SH = gu.oracle_scales(g, Ur, Vr, p, eps)
    _, S_RH, S_MG = gu.riemannian_scales(Ur, Vr, SG, SH)
    tau = gu.TOLS[dtype]["tau"]
    if gu.gram_in_edge_pass(k, dtype):  # rhvp's MG from U^T L and U^T phi, rhess's from U^T G
        assert gu.ew(MG2.cpu().numpy(), MG.cpu().numpy(), S_MG) <= 2 * tau
    else:
        assert torch.equal(MG, MG2)
    a, b = RH.double().cpu().numpy(), RH2.double().cpu().numpy()
    e = dict(vs_oracle=gu.ew(b, RHo, S_RH), vs_rhvp=gu.ew(b, a, S_RH), rel=gu.rel(b, RHo))
    print(e)
    assert e["vs_oracle"] <= tau and e["vs_rhvp"] <= 2 * tau and e["rel"] <= gu.TOLS[dtype]["norm"], e


def test_rhess_rejects_bad_arguments():
    g = gen.sbm_bernoulli(1000, 4, 0.05, 0.002)
    dg = gu.device_graph(g, 4)
    U = torch.randn(g.n, 4, device="cuda")
    V = torch.randn(g.n, 4, device="cuda")
    G = torch.randn(g.n, 4, device="cuda")
    with pytest.raises(pspec.PSpecError):
        pspec.rhess(dg, U, V, G, 1.5, 1e-8, RH=G)  # output overlaps the given gradient
    with pytest.raises(pspec.PSpecError):
        pspec.rhess(dg, U, V, G[:500], 1.5, 1e-8)  # G of the wrong shape
