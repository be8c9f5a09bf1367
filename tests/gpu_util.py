"""Helpers shared by the GPU parity tests: run the HIP path and the FP64 oracle on the same inputs.

Parity protocol: inputs are drawn in FP64, rounded to FP32 once, and both sides see those
rounded values (the oracle promoted exactly to FP64), so the difference measures the kernels'
arithmetic, not input rounding.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle as orc
from paper_2605_26975_amd import gen
from paper_2605_26975_amd import pspec


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def inputs(n, k, seed_u=gen.SEED_U, seed_v=gen.SEED_V):
    U = gen.block(n, k, seed_u)
    V = gen.block(n, k, seed_v)
    return U, V


def device_graph(g, k_max, weight_dtype=torch.float32):
    return pspec.Graph.from_host(g, "cuda", k_max=k_max, weight_dtype=weight_dtype)


def gpu_hvp(dg, U, V, p, eps, dtype, layout="separate"):
    """layout: "separate" (two n x k arrays) or "interleaved" (halves of one n x 2k array)."""
    if layout == "interleaved":
        k = U.shape[1]
        P = torch.empty((U.shape[0], 2 * k), dtype=dtype, device="cuda")
        P[:, :k] = torch.as_tensor(U).to(dtype)
        P[:, k:] = torch.as_tensor(V).to(dtype)
        Ut, Vt = P[:, :k], P[:, k:]
    else:
        Ut = torch.as_tensor(U).to(dtype).cuda()
        Vt = torch.as_tensor(V).to(dtype).cuda()
    HV, G, Fc = pspec.hvp(dg, Ut, Vt, p, eps)
    torch.cuda.synchronize()
    return HV.double().cpu().numpy(), G.double().cpu().numpy(), Fc.cpu().numpy()


def gpu_objective(dg, U, p, dtype):
    Ut = torch.as_tensor(U).to(dtype).cuda()
    F, Fc = pspec.objective(dg, Ut, p)
    torch.cuda.synchronize()
    return float(F.cpu()), Fc.cpu().numpy()


def oracle_hvp(g, U, V, p, eps):
    o = orc.default()
    return o.hvp(g.rowptr, g.col, g.w.astype(np.float64), U.astype(np.float64), V.astype(np.float64), p, eps)


def compare(g, k, p, eps, dtype, U=None, V=None, dg=None, layout="separate"):
    """Errors of the GPU path against the oracle: dict with F, Fcol (max rel), G, HV (Frobenius rel)."""
    if U is None:
        U, V = inputs(g.n, k)
    if dg is None:
        dg = device_graph(g, k)
    HVg, Gg, Fcg = gpu_hvp(dg, U, V, p, eps, dtype, layout)
    HVo, Go, Fco = oracle_hvp(g, U, V, p, eps)
    Fg, Fcg2 = gpu_objective(dg, U, p, dtype)
    err = dict(
        F=abs(Fg - Fco.sum()) / abs(Fco.sum()),
        Fcol=float(np.max(np.abs(Fcg - Fco) / np.abs(Fco))),
        G=rel(Gg, Go),
        HV=rel(HVg, HVo),
        G_colmax=max(rel(Gg[:, c], Go[:, c]) for c in range(k)),
        HV_colmax=max(rel(HVg[:, c], HVo[:, c]) for c in range(k)),
    )
    err["objective_matches_hvp"] = bool(np.array_equal(Fcg, Fcg2))
    return err
