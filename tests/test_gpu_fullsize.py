"""GPU parity at the full sizes of the five workloads, in the benchmark's launch configuration
(U and V as the two halves of one n x 2k array), against the FP64 oracle on every output.

Each case generates its graph, runs the oracle over all edges (multi-threaded; tens of seconds
for the largest) and bounds, for the FP32 fused path and the FP64 plain path, every entry of G and
HV by its forward-error scale, F relative, and G and HV relative over the block and per column
(tests/gpu_util.py).
"""
import numpy as np
import pytest
import torch

from paper_2605_26975_amd import gen, pspec
from tests import gpu_util as gu

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.mark.parametrize("name", ["knn100k", "grid128", "sbm8m", "rmat22"])
def test_fullsize_vs_oracle(name):
    cfg = gen.CONFIGS[name]
    k, p, eps = cfg["k"], cfg["p"][0], cfg["eps"]
    print(f"[case] fullsize {name} k={k} p={p}: generating", flush=True)
    g = cfg["graph"]()
    U, V = gu.inputs(g.n, k)
    dg = gu.device_graph(g, k)
    info = dg.info()
    print(f"[case] fullsize {name}: n={g.n} nnz={g.nnz} schedule={info}; oracle", flush=True)
    HVo, Go, Fco = gu.oracle_hvp(g, U, V, p, eps)
    print(f"[case] fullsize {name}: error scales", flush=True)
    SG, SH = gu.oracle_scales(g, U, V, p, eps)
    for dtype in (torch.float32, torch.float64):
        print(f"[case] fullsize {name}: {dtype}", flush=True)
        HV, G, Fc = gu.gpu_hvp(dg, U, V, p, eps, dtype, layout="interleaved")
        e = gu.errors(HV, G, Fc, HVo, Go, Fco, SG, SH)
        print(f"{name} {dtype}:", end=" ")
        gu.check(e, dtype)
        del HV, G
    # the fused Riemannian call against the unfused sequence at full size: bit for bit, or within
    # 2 tau entry by entry where the Gram products are formed in the edge pass
    P = torch.empty((g.n, 2 * k), dtype=torch.float32, device="cuda")
    P[:, :k] = torch.as_tensor(U)
    P[:, k:] = torch.as_tensor(V)
    Ut, Vt = P[:, :k], P[:, k:]
    RH, RG, MG, _ = pspec.rhvp(dg, Ut, Vt, p, eps)
    HV, G, _ = pspec.hvp(dg, Ut, Vt, p, eps)
    RG2, MG2 = pspec.project(Ut, G)
    RH2, _ = pspec.project(Ut, HV, X=Vt, MX=MG2)
    Uh, Vh = Ut.double().cpu().numpy(), Vt.double().cpu().numpy()
    S_RG, S_RH, S_MG = gu.riemannian_scales(Uh, Vh, SG, SH)
    tau = gu.TOLS[torch.float32]["tau"]
    if gu.gram_in_edge_pass(k, torch.float32):
        for nm, a, b, S in (("RG", RG, RG2, S_RG), ("RH", RH, RH2, S_RH), ("MG", MG, MG2, S_MG)):
            d = gu.ew(a.double().cpu().numpy(), b.double().cpu().numpy(), S)
            print(f"{name}: rhvp vs unfused {nm} element-wise {d:.2e}", flush=True)
            assert d <= 2 * tau, nm
    else:
        assert torch.equal(RG, RG2) and torch.equal(MG, MG2) and torch.equal(RH, RH2)
    # the fixed-U call of the truncated-CG loop: same F_col, MG and RH within the element-wise bound
    # of rhvp's (the scale of G and HV carried through the two Gram products)
    RH3, MG3, _ = pspec.rhess(dg, Ut, Vt, G, p, eps)
    torch.cuda.synchronize()
    if gu.gram_in_edge_pass(k, torch.float32):
        assert gu.ew(MG3.cpu().numpy(), MG.cpu().numpy(), S_MG) <= 2 * tau
    else:
        assert torch.equal(MG, MG3)
    d = gu.ew(RH3.double().cpu().numpy(), RH.double().cpu().numpy(), S_RH)
    print(f"{name}: rhess vs rhvp element-wise {d:.2e}", flush=True)
    assert d <= 2 * tau
    del P, RH, RG, HV, G, RG2, RH2, RH3
    if name == "rmat22":
        assert info["heavy_rows"] > 0 and info["split_rows"] > 0
        HV, G, Fc = gu.gpu_hvp(dg, U, V, p, eps, torch.float32, layout="separate")
        gu.check(gu.errors(HV, G, Fc, HVo, Go, Fco, SG, SH), torch.float32)
