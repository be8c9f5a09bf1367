#!/usr/bin/env python3
"""Benchmark of the p-Laplacian hot path on one MI355X.

Workload (default): stochastic block model with n = 8,000,000 nodes in 16 equal blocks with
block-contiguous ids, 43.2 M intra-block and 4.8 M inter-block edge draws (mean degree 12,
~96 M stored nonzeros), weights U[0.5, 1.5); k = 16 columns, p = 1.1, eps = 1e-8; U, V ~ N(0, 1)
in FP32.  Everything is synthetic and generated here from fixed seeds.

One step = one pass of the whole hot path:
  pspec_hvp       fused gradient + Hessian-vector product (edge pass, FP64 reductions, epilogue)
  pspec_project   Riemannian gradient  P_U(G)            (M_G = U^T G)
  pspec_project   Riemannian Hessian   P_U(HV) - V M_G
  pspec_retract   qf(U - t P_U(G))    (Cholesky-QR)
  pspec_objective F_p at the retracted point
`value` counts nnz * k edge-column updates per step (the gradient+HVP pass only) over the time of
the whole step.  The roofline object describes the fused edge kernel alone, timed with HIP events
that the library records around its edge pass on the call's stream.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "p-Laplacian grad+HVP edge·col updates/s, FP32 vs FP64, % HBM peak"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "edge_hvp_sbm8m_traffic.json")
VALU_FILE = os.path.join(PROFILES, "edge_hvp_sbm8m_valu.json")
VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_VALU_FLOPS_FP32_TRANS", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_SALU",
                 "SQ_INSTS_LDS", "SQ_BUSY_CU_CYCLES")
CUS, CLOCK_HZ = 256, 2.4e9  # MI355X compute units and peak engine clock
EDGE_KERNEL = "edge_light<float, float, 16, 2>"  # the fused grad+HVP edge pass at k = 16
COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read and 1 GiB written
WORKLOADS = {
    "sbm8m": "sbm8m: SBM n=8,000,000, 16 blocks, mean degree 12, w~U[0.5,1.5], k=16, p=1.1, eps=1e-8",
    "rmat22": "rmat22: R-MAT scale 22, edge factor 16, (0.57,0.19,0.19), w~U[0.1,1], k=32, p=1.05, eps=1e-8",
    "grid128": "grid128: 3-D 6-neighbour grid 128^3, unit weights, k=8, p=1.2, eps=1e-8",
    "knn100k": "knn100k: 10-NN of a 2-D 8-component Gaussian mixture, 100k points, k=8, p=1.3, eps=1e-8",
    "sbm1000": "sbm1000: SBM n=1000, 4 blocks, p_in 0.05, p_out 0.002, k=4, p=1.1, eps=1e-8",
}


def edge_source_hash() -> str:
    """Hash of the code (comments and whitespace removed) of the sources that define the fused edge
    kernel: the stored traffic figures go stale when that code changes."""
    h = hashlib.sha256()
    for f in ("edge.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2605_26975_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("".join(text.split()).encode())
    return h.hexdigest()[:16]


def algorithmic_edge_bytes(n: int, nnz: int, k: int, es: int = 4) -> int:
    """Fused edge pass, every input read once and every output written once:
    CSR (col + w per nonzero, rowptr per row), U and V read, raw L and J rows written."""
    return nnz * (4 + es) + (n + 1) * 8 + n * k * es * 4


def stored_traffic(workload: str, layout: str):
    """HBM bytes per launch of the edge kernel from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != edge_source_hash() or t.get("workload") != workload or t.get("layout") != layout:
        return None
    return t.get("bytes_per_launch")


def stored_valu(workload: str, layout: str, edge_ms: float):
    """The VALU ceiling of the edge kernel from the committed counter summary (same source check as
    the traffic): issue time of its VALU instructions (a wave64 instruction occupies a 16-lane SIMD
    for 4 cycles; 4 SIMDs per CU; transcendentals counted at full rate, so a lower bound) against
    the measured launch time, and the measured VALU busy fraction."""
    try:
        with open(VALU_FILE) as f:
            v = json.load(f)
    except (OSError, ValueError):
        return None
    if v.get("source_hash") != edge_source_hash() or v.get("workload") != workload or v.get("layout") != layout:
        return None
    ceiling_ms = v["valu_issue_ms"]
    return {"bound": "alu", "valu_issue_ms": ceiling_ms, "frac": ceiling_ms / edge_ms,
            "valu_busy": v["valu_busy"], "valu_insts_per_edge_col": v["valu_insts_per_edge_col"]}


def summarize_valu(pmc_dir: str, cmd: str, nnz: int, k: int) -> None:
    """Write the VALU summary of the edge kernel from one rocprofv3 --pmc run of VALU_COUNTERS."""
    import statistics

    rows = _csv_rows(os.path.join(pmc_dir, "**", "*counter_collection.csv"))
    is_edge = lambda nm: EDGE_KERNEL in nm.replace("pspec::(anonymous namespace)::", "")  # noqa: E731
    med = {}
    durs = {}
    for r in rows:
        if not is_edge(r["kernel_name"]):
            continue
        med.setdefault(r["counter_name"], []).append(float(r["counter_value"]))
        durs[r["dispatch_id"]] = (float(r["end_timestamp"]) - float(r["start_timestamp"])) * 1e-6
    med = {c: statistics.median(v) for c, v in med.items()}
    dur_ms = statistics.median(durs.values())
    valu = med["SQ_INSTS_VALU"]  # wave64 instructions, summed over the SIMDs of every SE
    # issue cycles per CU: 4 cycles per wave64 VALU instruction on one of its 4 SIMDs
    issue_ms = valu * 4 / 4 / CUS / CLOCK_HZ * 1e3
    # rocprofv3's VALUBusy: SQ_ACTIVE_INST_VALU (quad-cycles summed over SIMDs) / CUs / cycles
    busy = med["SQ_ACTIVE_INST_VALU"] / CUS / (CLOCK_HZ * dur_ms * 1e-3)
    out = {
        "workload": "sbm8m", "layout": "interleaved", "kernel": EDGE_KERNEL, "source_hash": edge_source_hash(),
        "counters_per_dispatch": med, "dispatch_ms_under_counters": dur_ms,
        "valu_insts_per_edge_col": valu * 64 / (nnz * k), "valu_issue_ms": issue_ms, "valu_busy": busy,
        "command": cmd,
    }
    with open(VALU_FILE, "w") as f:
        json.dump(out, f, indent=1)
    md = ["# VALU work of the fused grad+HVP edge pass: SBM n=8,000,000, k=16, FP32", "",
          "Counter run (from the repository root, one MI355X):", "", "```", cmd, "```", "",
          "| quantity | value |", "|---|---|"]
    md += [f"| {c} (per dispatch, median) | {v:.6g} |" for c, v in med.items()]
    md += [f"| dispatch time under counters (ms) | {dur_ms:.4g} |",
           f"| VALU lane-instructions per edge-col | {out['valu_insts_per_edge_col']:.4g} |",
           f"| VALU issue time at {CUS} CUs x {CLOCK_HZ / 1e9:.1f} GHz, all at full rate (ms) | {issue_ms:.4g} |",
           f"| VALU busy (rocprofv3 VALUBusy: SQ_ACTIVE_INST_VALU / CUs / cycles) | {busy:.3f} |", "",
           "SQ_INSTS_VALU_FLOPS_FP32_TRANS reads 0.04 per edge-col where the kernel issues one v_log_f32 and "
           "one v_exp_f32 per edge-col: that counter does not count them here, so the issue time takes "
           "every VALU instruction at full rate (a lower bound; the two transcendentals run at quarter rate)."]
    with open(os.path.join(PROFILES, "edge_hvp_sbm8m_valu.md"), "w") as f:
        f.write("\n".join(md) + "\n")


class HipEvents:
    """Raw hipEvent_t pairs from the HIP runtime torch already loaded (the library records them)."""

    def __init__(self, count: int):
        import ctypes

        self.ct = ctypes
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.pairs = []
        for _ in range(count):
            a, b = ctypes.c_void_p(), ctypes.c_void_p()
            if self.hip.hipEventCreate(ctypes.byref(a)) or self.hip.hipEventCreate(ctypes.byref(b)):
                raise RuntimeError("hipEventCreate failed")
            self.pairs.append((a, b))

    def elapsed_ms(self, i: int) -> float:
        ms = self.ct.c_float()
        a, b = self.pairs[i]
        if self.hip.hipEventElapsedTime(self.ct.byref(ms), a, b):
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def close(self):
        for a, b in self.pairs:
            self.hip.hipEventDestroy(a)
            self.hip.hipEventDestroy(b)


def _csv_rows(pattern):
    import csv
    import glob

    rows = []
    for f in sorted(glob.glob(pattern, recursive=True)):
        with open(f) as fh:
            rows.extend({k.lower(): v for k, v in r.items()} for r in csv.DictReader(fh))
    return rows


def summarize_profile(trace_dir: str, fetch_dir: str, write_dir: str, cmd_trace: str, cmd_fetch: str,
                      cmd_write: str) -> None:
    """Write the committed profile summaries from rocprofv3 CSV output (kernel stats and the
    FETCH_SIZE / WRITE_SIZE counter runs)."""
    import statistics

    stats = _csv_rows(os.path.join(trace_dir, "**", "*kernel_stats.csv"))
    lines = ["# Kernel trace: SBM n=8,000,000, k=16, p=1.1, FP32, interleaved U|V", "",
             "Command (from the repository root, on one MI355X):", "", "```", cmd_trace, "```", "",
             "| kernel | calls | average us | share % |", "|---|---|---|---|"]
    for r in stats[:14]:
        name = r["name"].replace("pspec::(anonymous namespace)::", "")
        name = name.split("(")[0][:80]
        lines.append(f"| `{name}` | {r['calls']} | {float(r['averagens']) / 1e3:.1f} | {float(r['percentage']):.1f} |")
    with open(os.path.join(PROFILES, "edge_hvp_sbm8m_kernel_trace.md"), "w") as f:
        f.write("\n".join(lines) + "\n")

    def per_dispatch(rows, counter, pred):
        vals = [float(r["counter_value"]) for r in rows if r["counter_name"] == counter and pred(r["kernel_name"])]
        return statistics.median(vals) if vals else None

    fetch = _csv_rows(os.path.join(fetch_dir, "**", "*counter_collection.csv"))
    write = _csv_rows(os.path.join(write_dir, "**", "*counter_collection.csv"))
    is_edge = lambda nm: EDGE_KERNEL in nm.replace("pspec::(anonymous namespace)::", "")  # noqa: E731
    is_copy = lambda nm: "axpby_k<float, 16, true>" in nm  # the calibration copy (bench.py --copy-calibration)
    f_edge = per_dispatch(fetch, "FETCH_SIZE", is_edge)
    w_edge = per_dispatch(write, "WRITE_SIZE", is_edge)
    f_copy = per_dispatch(fetch, "FETCH_SIZE", is_copy)
    w_copy = per_dispatch(write, "WRITE_SIZE", is_copy)
    kib = COPY_BYTES / 1024.0
    f_scale = kib / f_copy if f_copy else None
    w_scale = kib / w_copy if w_copy else None
    traffic = None
    if f_edge is not None and w_edge is not None and f_scale and w_scale:
        traffic = (f_edge * f_scale + w_edge * w_scale) * 1024.0
    out = {
        "workload": "sbm8m",
        "layout": "interleaved",
        "kernel": EDGE_KERNEL,
        "source_hash": edge_source_hash(),
        "fetch_kib_per_dispatch": f_edge,
        "write_kib_per_dispatch": w_edge,
        "copy_fetch_kib": f_copy,
        "copy_write_kib": w_copy,
        "fetch_scale": f_scale,
        "write_scale": w_scale,
        "bytes_per_launch": traffic,
        "commands": [cmd_fetch, cmd_write],
    }
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    alg = None
    md = ["# HBM traffic of the fused grad+HVP edge pass: SBM n=8,000,000, k=16, FP32", "",
          "Counter runs (from the repository root, one MI355X, one counter block per run):", "", "```",
          cmd_fetch, cmd_write, "```", "",
          f"A plain device copy of {COPY_BYTES >> 20} MiB (read and written once) calibrates each counter: "
          f"scale = known KiB / counted KiB.", "",
          "| quantity | value |", "|---|---|",
          f"| FETCH_SIZE, edge kernel (KiB/dispatch, median) | {f_edge} |",
          f"| WRITE_SIZE, edge kernel (KiB/dispatch, median) | {w_edge} |",
          f"| FETCH_SIZE, copy (KiB) | {f_copy} |", f"| WRITE_SIZE, copy (KiB) | {w_copy} |",
          f"| fetch scale | {f_scale} |", f"| write scale | {w_scale} |",
          f"| HBM bytes per launch (scaled) | {traffic} |"]
    with open(os.path.join(PROFILES, "edge_hvp_sbm8m_traffic.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    del alg


def cpu_baseline(g, U_h, V_h, k: int, p: float, eps: float, workload: str):
    """Time the FP64 oracle (as it stands) for one grad+HVP call on the benchmarked graph and block,
    on every host core; and single-threaded on a bounded sample of the same workload (the rows of the
    first SBM block and the edges among them, the induced subgraph: ~1/16 of the graph)."""
    import numpy as np

    import oracle
    from paper_2605_26975_amd import gen

    o = oracle.default()
    U = U_h.astype(np.float64)
    V = V_h.astype(np.float64)
    w = g.w.astype(np.float64)
    t0 = time.perf_counter()
    o.hvp(g.rowptr, g.col, w, U, V, p, eps)
    dt = time.perf_counter() - t0
    cores = o.num_threads()
    # single thread on the first block (block-contiguous ids: rows [0, n / 16))
    keep = np.zeros(g.n, dtype=bool)
    keep[: g.n // 16] = True
    sub, old = gen.induced(g, keep)
    o.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        o.hvp(sub.rowptr, sub.col, sub.w.astype(np.float64), U[old], V[old], p, eps)
        dt1 = time.perf_counter() - t1
    finally:
        o.set_num_threads(cores)
    return {
        "value": g.nnz * k / dt,
        "unit": "edge*col updates/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"one FP64 oracle grad+HVP call on the full {workload} graph and block (n={g.n}, nnz={g.nnz}, "
                  f"k={k}, p={p}): {dt:.2f} s on {cores} threads",
        "single_thread": {
            "value": sub.nnz * k / dt1, "unit": "edge*col updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one FP64 oracle grad+HVP call, 1 thread, on the subgraph induced by the first block "
                      f"(n={sub.n}, nnz={sub.nnz}, k={k}, p={p}): {dt1:.2f} s",
        },
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sbm8m", choices=["sbm8m", "rmat22", "grid128", "knn100k", "sbm1000"],
                    help="the headline is sbm8m; the others are reported for load balance and context")
    ap.add_argument("--layout", default="interleaved", choices=["interleaved", "separate"],
                    help="U and V as the two halves of one n x 2k array, or two n x k arrays")
    ap.add_argument("--step", default="fused", choices=["fused", "unfused"],
                    help="fused: one pspec_rhvp call for the Riemannian gradient and Hessian; unfused: pspec_hvp "
                         "and two pspec_project calls (identical results)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--permute", action="store_true",
                    help="relabel the nodes by a seeded random permutation first (node-order sensitivity line)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the side measurements (per-call times, cold edge pass, streaming-read rate)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration for profiles)")
    ap.add_argument("--summarize-valu", nargs=4, metavar=("PMC_DIR", "CMD", "NNZ", "K"),
                    help="write the VALU counter summary of the edge kernel and exit")
    ap.add_argument("--summarize-profile", nargs=6, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR", "CMD_TRACE",
                                                            "CMD_FETCH", "CMD_WRITE"),
                    help="write the profiles/ summaries from rocprofv3 CSV output and exit (no GPU needed)")
    args = ap.parse_args()
    if args.summarize_valu:
        summarize_valu(args.summarize_valu[0], args.summarize_valu[1], int(args.summarize_valu[2]),
                       int(args.summarize_valu[3]))
        return 0
    if args.summarize_profile:
        summarize_profile(*args.summarize_profile)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE={world}); run it with --gpus 1.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2605_26975_amd import gen, pspec

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = gen.CONFIGS[args.workload]
    k, p, eps = cfg["k"], cfg["p"][-1], cfg["eps"]
    t0 = time.perf_counter()
    g = cfg["graph"]()
    if args.permute:
        g = gen.permute(g, seed=7)
    print(f"[bench] graph n={g.n} nnz={g.nnz} generated in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
          flush=True)
    U_h = gen.block(g.n, k, gen.SEED_U)
    V_h = gen.block(g.n, k, gen.SEED_V)
    dg = pspec.Graph.from_host(g, dev, k_max=k)
    n, nnz = g.n, g.nnz
    keep_host_graph = not args.no_cpu_baseline and args.workload == "sbm8m"
    if not keep_host_graph:
        del g

    def make_inputs(dtype):
        if args.layout == "interleaved":
            P = torch.empty((n, 2 * k), dtype=dtype, device=dev)
            P[:, :k] = torch.as_tensor(U_h).to(dtype)
            P[:, k:] = torch.as_tensor(V_h).to(dtype)
            return P[:, :k], P[:, k:], P
        U = torch.as_tensor(U_h).to(dtype).to(dev)
        V = torch.as_tensor(V_h).to(dtype).to(dev)
        return U, V, None

    def run(dtype, steps, warmup, timed_kernel=True):
        U, V, keep = make_inputs(dtype)
        unfused = args.step != "fused"
        HV = torch.empty((n, k), dtype=dtype, device=dev) if unfused else None
        G = torch.empty((n, k), dtype=dtype, device=dev) if unfused else None
        RG = torch.empty((n, k), dtype=dtype, device=dev)
        RH = torch.empty((n, k), dtype=dtype, device=dev)
        Un = torch.empty((n, k), dtype=dtype, device=dev)
        MG = torch.empty((k, k), dtype=torch.float64, device=dev)
        Fc = torch.empty(k, dtype=torch.float64, device=dev)
        F = torch.empty((), dtype=torch.float64, device=dev)
        Fc2 = torch.empty(k, dtype=torch.float64, device=dev)
        t_step = -1e-3

        def step(pair=None):
            # Riemannian gradient and Hessian applied to V (edge pass, epilogue, Gram matrices and
            # projections), a retraction along the Riemannian gradient, the objective there
            if pair is not None:
                dg.set_timing_events_raw(*pair)
            if args.step == "fused":
                pspec.rhvp(dg, U, V, p, eps, RH=RH, RG=RG, MG=MG, F_col=Fc)
            else:
                pspec.hvp(dg, U, V, p, eps, HV=HV, G=G, F_col=Fc)
            if pair is not None:
                dg.set_timing_events_raw(None, None)
            if args.step != "fused":
                pspec.project(U, G, out=RG, M=MG)
                pspec.project(U, HV, X=V, MX=MG, out=RH)
            pspec.retract(U, RG, t_step, out=Un)
            pspec.objective(dg, Un, p, F_col=Fc2, F=F)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        evs = HipEvents(steps)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for i in range(steps):
            step(evs.pairs[i] if timed_kernel else None)
        stop.record()
        torch.cuda.synchronize()
        total_ms = start.elapsed_time(stop)
        edge_ms = [evs.elapsed_ms(i) for i in range(steps)] if timed_kernel else []
        evs.close()
        ok = bool(torch.isfinite(F).item()) and bool(torch.isfinite(RH).all().item())
        return total_ms / steps, edge_ms, ok

    def extras(reps: int = 10):
        """FP32 side measurements (not the metric): each call of the step on its own, the unfused
        pspec_hvp call (edge pass + epilogue), one k-means step on U's rows (k clusters) with its
        algorithmic rate, the edge pass with the Infinity Cache flushed before every run, and a
        streaming-read reference rate of this GPU (pspec_dot over 2 GiB)."""
        dtype = torch.float32
        U, V, keep = make_inputs(dtype)
        RG, RH, Un, HV, G = (torch.empty((n, k), dtype=dtype, device=dev) for _ in range(5))
        MG = torch.empty((k, k), dtype=torch.float64, device=dev)
        Fc = torch.empty(k, dtype=torch.float64, device=dev)
        F = torch.empty((), dtype=torch.float64, device=dev)
        # one Lloyd step of the k-means discretisation of U's rows into k clusters (labels written)
        Ck = U[:k].double().contiguous()
        lab = torch.empty(n, dtype=torch.int32, device=dev)
        st = torch.empty((k, k + 2), dtype=torch.float64, device=dev)
        calls = {
            "rhvp": lambda: pspec.rhvp(dg, U, V, p, eps, RH=RH, RG=RG, MG=MG, F_col=Fc),
            "hvp": lambda: pspec.hvp(dg, U, V, p, eps, HV=HV, G=G, F_col=Fc),
            "project": lambda: pspec.project(U, G, out=RG, M=MG),
            "retract": lambda: pspec.retract(U, RG, -1e-3, out=Un),
            "objective": lambda: pspec.objective(dg, Un, p, F_col=Fc, F=F),
            "kmeans_step": lambda: pspec.kmeans_step(U, Ck, labels=lab, stats=st),
        }
        ms = {}
        for name, fn in calls.items():
            fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                fn()
            b.record()
            torch.cuda.synchronize()
            ms[name] = a.elapsed_time(b) / reps
        # the gather floor: the same edge pass with its arithmetic replaced by a sum of the gathered
        # values (same kernels, grid, loads and stores), timed by the same events
        evs = HipEvents(reps)
        pspec.hvp_gather_floor(dg, U, V, HV=HV, G=G)
        for i in range(reps):
            dg.set_timing_events_raw(*evs.pairs[i])
            pspec.hvp_gather_floor(dg, U, V, HV=HV, G=G)
            dg.set_timing_events_raw(None, None)
        torch.cuda.synchronize()
        floor = [evs.elapsed_ms(i) for i in range(reps)]
        evs.close()
        # edge pass with a cold Infinity Cache: 512 MiB written before every run
        flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
        evs = HipEvents(reps)
        for i in range(reps):
            flush.zero_()
            dg.set_timing_events_raw(*evs.pairs[i])
            calls["hvp"]()
            dg.set_timing_events_raw(None, None)
        torch.cuda.synchronize()
        cold = [evs.elapsed_ms(i) for i in range(reps)]
        evs.close()
        del flush
        # streaming read: sum_ij A_ij B_ij over two 1 GiB blocks
        rows = (1 << 30) // (16 * 4)
        A = torch.ones((rows, 16), dtype=dtype, device=dev)
        B = torch.ones((rows, 16), dtype=dtype, device=dev)
        pspec.dot(A, B)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            pspec.dot(A, B)
        b.record()
        torch.cuda.synchronize()
        read_gbs = 2 * (1 << 30) / (a.elapsed_time(b) / reps * 1e-3) / 1e9
        del A, B
        return {
            "call_ms": ms,
            "hvp_call_value": nnz * k / (ms["hvp"] * 1e-3),
            "edge_pass_cold_ms": float(np.mean(cold)),
            "gather_floor_ms": float(np.mean(floor)),
            "kmeans_step_GBps": (n * k * U.element_size() + 4 * n) / (ms["kmeans_step"] * 1e-3) / 1e9,
            "read_stream_GBps": read_gbs,
        }

    if args.copy_calibration:
        # Y <- 1 * X + 0 * Y through the library's axpby: reads X once, writes Y once (a plain copy)
        src = torch.ones((COPY_BYTES // 64, 16), dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            pspec.axpby(1.0, src, 0.0, dst)
        torch.cuda.synchronize()
        del src, dst
    t32, edge32, ok32 = run(torch.float32, args.steps, args.warmup)
    print(f"[bench] fp32 step {t32:.3f} ms, edge pass {np.mean(edge32):.3f} ms", file=sys.stderr, flush=True)
    more = None if args.no_extras else extras()
    fp64 = None
    if not args.no_fp64:
        t64, edge64, ok64 = run(torch.float64, max(3, args.steps // 4), 1)
        fp64 = {
            "ms_per_step": t64,
            "value": nnz * k / (t64 * 1e-3),
            "edge_pass_ms": float(np.mean(edge64)),
            "edge_pass_value": nnz * k / (np.mean(edge64) * 1e-3),
            "finite": ok64,
        }
        print(f"[bench] fp64 step {t64:.3f} ms, edge pass {np.mean(edge64):.3f} ms", file=sys.stderr, flush=True)

    edge_ms = float(np.mean(edge32))
    alg_bytes = algorithmic_edge_bytes(n, nnz, k)
    achieved = alg_bytes / (edge_ms * 1e-3) / 1e9
    traffic = None if args.permute else stored_traffic(args.workload, args.layout)
    out = {
        "metric": METRIC,
        "value": nnz * k / (t32 * 1e-3),
        "unit": "edge*col updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.workload],
            "n": n,
            "nnz": nnz,
            "k": k,
            "p": p,
            "eps": eps,
            "layout": args.layout,
            "node_order": "random permutation (seed 7)" if args.permute else "generator order",
            "step": ("rhvp (grad, HVP, both Grassmann projections)" if args.step == "fused" else
                     "hvp (fused grad) + 2x project") + " + retract + objective",
            "edge_col_updates_per_step": nnz * k,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "fused grad+HVP edge pass (light rows, heavy chunks, split-row combine)",
            "algorithmic_bytes_per_launch": alg_bytes,
            "launch_ms": edge_ms,
            "valu": None if args.permute else stored_valu(args.workload, args.layout, edge_ms),
        },
        "edge_pass_value": nnz * k / (edge_ms * 1e-3),
        "measurements": None if more is None else dict(
            more, edge_frac_of_read_stream=achieved / more["read_stream_GBps"],
            edge_frac_of_gather_floor=more["gather_floor_ms"] / edge_ms),
        "fp64": fp64,
        "speedup_fp32_over_fp64": (fp64["ms_per_step"] / t32) if fp64 else None,
        "finite": ok32,
    }
    if keep_host_graph:
        print("[bench] timing the CPU oracle on the same workload ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(g, U_h, V_h, k, p, eps, args.workload)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
