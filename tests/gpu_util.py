"""Helpers shared by the GPU parity tests: run the HIP path and the FP64 oracle on the same inputs
and bound every entry of the difference.

Parity protocol: inputs are drawn in FP64, rounded to FP32 once, and both sides see those
rounded values (the oracle promoted exactly to FP64), so the difference measures the kernels'
arithmetic, not input rounding.

Element-wise bound.  Every entry x of G and HV is a signed sum of terms; the oracle's
``error_scales`` returns its forward-error scale S, the same sum over absolute values with each
power term weighted by its conditioning.  Any evaluation whose elementary operations carry a
relative error r agrees with the exact value to (c + m) r S, m being the longest sequential sum, so
the tests assert |x_gpu - x_oracle| <= tau S for EVERY entry.  tau = 4e-6 (34 units of 2^-23) for
the FP32 path and 1e-13 for the FP64 path: the largest ratios measured over every parity case,
full-size R-MAT (FP32 sums of up to 256 terms per lane) included, are 5e-7 and 3.2e-15, so the
bounds leave a margin of about 8x and 30x and still catch one dropped edge term in a row of up to
~2e5 (FP32) edges.  On top of that F (relative) and the relative Frobenius error of G and HV over
the block and over every single column must stay below 1e-5 (FP32: the stated target; measured
<= 4.4e-8 for F, <= 2.1e-6 per column) and 1e-13 (FP64; measured <= 3.6e-15).
"""
from __future__ import annotations

import numpy as np
import torch

import oracle as orc
from paper_2605_26975_amd import gen
from paper_2605_26975_amd import pspec

TOLS = {
    torch.float32: dict(F=1e-5, norm=1e-5, tau=4e-6),
    torch.float64: dict(F=1e-13, norm=1e-13, tau=1e-13),
}


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def colmax(a, b) -> float:
    """Largest relative Frobenius error over the columns of an n x k block."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return max(rel(a[:, c], b[:, c]) for c in range(b.shape[1])) if b.ndim == 2 and b.shape[1] else rel(a, b)


def ew(a, b, S) -> float:
    """max over entries of |a - b| / S.  An entry with S = 0 must match exactly (else inf); NaN in
    either operand gives inf."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    d = np.abs(a - b)
    if not np.all(np.isfinite(d)):
        return float("inf")
    pos = S > 0
    if np.any(d[~pos] != 0):
        return float("inf")
    return float(np.max(d[pos] / S[pos])) if np.any(pos) else 0.0


def inputs(n, k, seed_u=gen.SEED_U, seed_v=gen.SEED_V):
    U = gen.block(n, k, seed_u)
    V = gen.block(n, k, seed_v)
    return U, V


def shuffled(g, seed=5):
    """The same graph with each row's entries in a seeded random order (columns no longer ascend)."""
    rng = np.random.default_rng(seed)
    key = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.rowptr)) * 2.0 + rng.random(g.nnz)
    order = np.argsort(key, kind="stable")
    return gen.Graph(g.n, g.rowptr.copy(), g.col[order].copy(), g.w[order].copy(), name=g.name + "-shuffled")


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


def oracle_scales(g, U, V, p, eps, sparse=False):
    o = orc.default()
    return o.error_scales(g.rowptr, g.col, g.w.astype(np.float64), U.astype(np.float64), V.astype(np.float64), p,
                          eps, sparse=sparse)


def gram_in_edge_pass(k, dtype) -> bool:
    """Whether pspec_rhvp / pspec_rhess form their Gram products inside the edge pass (FP32,
    9 <= k <= 16).
    Their MG and MH then come from U^T L, U^T J, U^T phi and U^T (psi v) combined in FP64, which
    agrees with the Gram products of the finalized G and HV (the unfused sequence) to rounding, not
    bit for bit."""
    return 9 <= k <= 16 and dtype == torch.float32


def riemannian_scales(U, V, SG, SH):
    """Element-wise scales of RG = G - U (U^T G), RH = HV - U (U^T HV) - V (U^T G) and MG = U^T G:
    the forward-error scales of G and HV carried through the products (U, V as FP64 arrays)."""
    aU, aV = np.abs(U), np.abs(V)
    MGs = aU.T @ SG
    return SG + aU @ MGs, SH + aU @ (aU.T @ SH) + aV @ MGs, MGs


def errors(HVg, Gg, Fcg, HVo, Go, Fco, SG, SH) -> dict:
    """Every error measure of one grad+HVP result against the oracle's."""
    return dict(
        Fcol=float(np.max(np.abs(Fcg - Fco) / np.abs(Fco))) if Fco.size else 0.0,
        G=rel(Gg, Go), HV=rel(HVg, HVo),
        G_colmax=colmax(Gg, Go), HV_colmax=colmax(HVg, HVo),
        G_ew=ew(Gg, Go, SG), HV_ew=ew(HVg, HVo, SH),
    )


def compare(g, k, p, eps, dtype, U=None, V=None, dg=None, layout="separate"):
    """Errors of the GPU path against the oracle (see errors(); plus F and F_col of pspec_objective,
    which on graphs with ascending rows sums each undirected edge once and so agrees with the HVP
    call's F_col to rounding only)."""
    if U is None:
        U, V = inputs(g.n, k)
    if dg is None:
        dg = device_graph(g, k)
    HVg, Gg, Fcg = gpu_hvp(dg, U, V, p, eps, dtype, layout)
    HVo, Go, Fco = oracle_hvp(g, U, V, p, eps)
    SG, SH = oracle_scales(g, U, V, p, eps)
    Fg, Fcg2 = gpu_objective(dg, U, p, dtype)
    err = errors(HVg, Gg, Fcg, HVo, Go, Fco, SG, SH)
    err["F"] = abs(Fg - Fco.sum()) / abs(Fco.sum())
    err["Fcol_obj"] = float(np.max(np.abs(Fcg2 - Fco) / np.abs(Fco))) if Fco.size else 0.0
    return err


def check(e: dict, dtype, norms=True) -> None:
    """Assert the parity bounds of TOLS[dtype] on an errors()/compare() dict (printed first).
    ``norms=False`` keeps the element-wise and F bounds only (for blocks near a stationary point,
    where G is a difference of nearly equal terms and its norm says nothing about the arithmetic)."""
    t = TOLS[dtype]
    print({k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in e.items()}, flush=True)
    assert e.get("F", 0.0) <= t["F"] and e["Fcol"] <= t["F"] and e.get("Fcol_obj", 0.0) <= t["F"], e
    if norms:
        assert e["G"] <= t["norm"] and e["G_colmax"] <= t["norm"], e
        assert e["HV"] <= t["norm"] and e["HV_colmax"] <= t["norm"], e
    assert e["G_ew"] <= t["tau"] and e["HV_ew"] <= t["tau"], e
