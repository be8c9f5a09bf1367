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
CUS, CLOCK_HZ = 256, 2.4e9  # MI355X compute units and peak engine clock
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


def _pad_k(k: int) -> int:
    K = 4
    while K < k:
        K *= 2
    return K


def _short(name: str) -> str:
    return name.replace("pspec::(anonymous namespace)::", "").replace("void ", "", 1).split("(")[0]


def is_edge_pass_kernel(name: str, k: int) -> bool:
    """The kernels of the FP32 grad+HVP edge pass at width k: light rows (at 9 <= k <= 16 with the
    Gram products), heavy chunks, split-row combine (not the gather-floor reference, whose FLOOR
    template argument is true)."""
    nm, K = _short(name), _pad_k(k)
    return (nm in (f"edge_light<float, float, {K}, 2, false, false>", f"edge_light<float, float, {K}, 2, false, true>")
            or (nm.startswith(f"edge_heavy<float, float, {K}, 2, ") and nm.endswith(", false>"))
            or nm == "combine_split<float, 2>")


def _stored(kind: str, workload: str, layout: str):
    try:
        with open(os.path.join(PROFILES, f"edge_hvp_{workload}_{kind}.json")) as f:
            v = json.load(f)
    except (OSError, ValueError):
        return None
    if v.get("source_hash") != edge_source_hash() or v.get("workload") != workload or v.get("layout") != layout:
        return None
    return v


def stored_traffic(workload: str, layout: str):
    """HBM bytes per edge pass (all its kernels) from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    v = _stored("traffic", workload, layout)
    return None if v is None else v.get("bytes_per_launch")


def stored_valu(workload: str, layout: str, edge_ms: float):
    """The VALU figures of the edge pass from the committed counter summary (same source check as the
    traffic): issue time of its VALU instructions (a wave64 instruction occupies a 16-lane SIMD for 4
    cycles, 4 SIMDs per CU; transcendentals at a quarter of the rate) against the measured pass, and
    the measured VALU busy fraction."""
    v = _stored("valu", workload, layout)
    if v is None:
        return None
    return {"bound": "alu", "valu_issue_ms": v["valu_issue_ms"], "frac": v["valu_issue_ms"] / edge_ms,
            "valu_busy": v["valu_busy"], "valu_insts_per_edge_col": v["valu_insts_per_edge_col"],
            "trans_insts_per_edge_col": v.get("trans_insts_per_edge_col")}


def _csv_rows(pattern):
    import csv
    import glob

    rows = []
    for f in sorted(glob.glob(pattern, recursive=True)):
        with open(f) as fh:
            rows.extend({k.lower(): v for k, v in r.items()} for r in csv.DictReader(fh))
    return rows


def _per_kernel(rows):
    """{kernel: {counter: median per dispatch}} and {kernel: median dispatch ms} from counter rows."""
    import statistics

    vals, durs = {}, {}
    for r in rows:
        nm = _short(r["kernel_name"])
        vals.setdefault(nm, {}).setdefault(r["counter_name"], []).append(float(r["counter_value"]))
        durs.setdefault(nm, {})[r["dispatch_id"]] = (float(r["end_timestamp"]) - float(r["start_timestamp"])) * 1e-6
    med = {nm: {c: statistics.median(v) for c, v in cs.items()} for nm, cs in vals.items()}
    ms = {nm: statistics.median(d.values()) for nm, d in durs.items()}
    return med, ms


def summarize_pmc(workload: str, nnz: int, k: int, out_name: str, runs: list) -> None:
    """Write profiles/<out_name>.md from rocprofv3 --pmc runs (each "DIR::COMMAND"): per-kernel medians
    of every counter for the edge-pass kernels, the Gram kernels and the calibration copy, and what
    follows from them -- HBM traffic per edge pass (FETCH_SIZE, WRITE_SIZE scaled by what they read
    for the 1 GiB copy; saved to edge_hvp_<workload>_traffic.json), VALU and transcendental
    instructions per edge-col (edge_hvp_<workload>_valu.json), L2 hit rates, FP64 matrix-core use."""
    med, ms = {}, {}
    cmds = []
    for run in runs:
        d, cmd = run.split("::", 1)
        cmds.append(cmd)
        m, t = _per_kernel(_csv_rows(os.path.join(d, "**", "*counter_collection.csv")))
        for nm, cs in m.items():
            med.setdefault(nm, {}).update(cs)
            ms[nm] = t[nm]
    edge = [nm for nm in med if is_edge_pass_kernel(nm, k)]
    gram = [nm for nm in med if nm.startswith(("finalize_gram", "gram_heavy", "sum_range", "apply_rhvp",
                                               "gram_partial", "apply_rows"))]
    copy = [nm for nm in med if nm.startswith("axpby_k<float, 16, true>")]
    layout, lines = "interleaved", []
    lines += [f"# Counters: {workload} (nnz = {nnz}, k = {k}), FP32", "",
              "Counter runs (from the repository root, one MI355X, one counter group per run):", "", "```"]
    lines += cmds + ["```", "", "Per-dispatch medians.", "", "| kernel | ms | counter | value |", "|---|---|---|---|"]
    for nm in edge + gram + copy:
        for c, v in sorted(med[nm].items()):
            lines.append(f"| `{nm[:70]}` | {ms[nm]:.4g} | {c} | {v:.6g} |")
    lines.append("")
    edge_ms = sum(ms[nm] for nm in edge)
    kib = COPY_BYTES / 1024.0
    have = lambda c, nms: all(c in med[nm] for nm in nms) and nms  # noqa: E731
    if have("FETCH_SIZE", edge) and have("WRITE_SIZE", edge) and copy and "FETCH_SIZE" in med[copy[0]] \
            and "WRITE_SIZE" in med[copy[0]]:
        fs, ws = kib / med[copy[0]]["FETCH_SIZE"], kib / med[copy[0]]["WRITE_SIZE"]
        fetch = sum(med[nm]["FETCH_SIZE"] for nm in edge)
        write = sum(med[nm]["WRITE_SIZE"] for nm in edge)
        traffic = (fetch * fs + write * ws) * 1024.0
        out = {"workload": workload, "layout": layout, "kernels": edge, "source_hash": edge_source_hash(),
               "fetch_kib_per_pass": fetch, "write_kib_per_pass": write, "fetch_scale": fs, "write_scale": ws,
               "bytes_per_launch": traffic, "commands": cmds}
        with open(os.path.join(PROFILES, f"edge_hvp_{workload}_traffic.json"), "w") as f:
            json.dump(out, f, indent=1)
        lines += [f"HBM traffic of the edge pass ({', '.join(f'`{e}`' for e in edge)}): FETCH_SIZE {fetch:.6g} KiB "
                  f"x {fs:.4f} + WRITE_SIZE {write:.6g} KiB x {ws:.4f} = {traffic / 1e9:.3f} GB per pass (the scales "
                  f"are known KiB / counted KiB of a plain 1 GiB device copy in the same runs); "
                  f"{traffic / (nnz * k):.3f} B per edge-col; {traffic / (edge_ms * 1e-3) / 1e9:.0f} GB/s over "
                  f"the pass's {edge_ms:.3f} ms under counters.", ""]
    if have("SQ_INSTS_VALU", edge):
        valu = sum(med[nm]["SQ_INSTS_VALU"] for nm in edge)
        trans = sum(med[nm].get("SQ_INSTS_VALU_TRANS_F32", 0.0) for nm in edge)
        # issue cycles per CU: 4 per wave64 VALU instruction on one of 4 SIMDs; transcendentals 4x that
        issue_ms = (valu + 3 * trans) * 4 / 4 / CUS / CLOCK_HZ * 1e3
        busy_num = sum(med[nm].get("SQ_ACTIVE_INST_VALU", 0.0) for nm in edge)
        busy = busy_num / CUS / (CLOCK_HZ * edge_ms * 1e-3)
        out = {"workload": workload, "layout": layout, "kernels": edge, "source_hash": edge_source_hash(),
               "valu_insts_per_edge_col": valu * 64 / (nnz * k), "trans_insts_per_edge_col": trans * 64 / (nnz * k),
               "valu_issue_ms": issue_ms, "valu_busy": busy, "dispatch_ms_under_counters": edge_ms, "commands": cmds}
        with open(os.path.join(PROFILES, f"edge_hvp_{workload}_valu.json"), "w") as f:
            json.dump(out, f, indent=1)
        lines += [f"VALU of the edge pass: {out['valu_insts_per_edge_col']:.3g} lane-instructions per edge-col, of "
                  f"which {out['trans_insts_per_edge_col']:.3g} transcendental (SQ_INSTS_VALU_TRANS_F32); issue time "
                  f"{issue_ms:.3f} ms at {CUS} CUs x {CLOCK_HZ / 1e9:.1f} GHz (transcendentals at quarter rate) "
                  f"against {edge_ms:.3f} ms; VALU busy (SQ_ACTIVE_INST_VALU / CUs / cycles) {busy:.2f}.", ""]
    for nm in edge + gram:
        cs = med[nm]
        if "TCC_HIT_sum" in cs and "TCC_MISS_sum" in cs:
            h, m = cs["TCC_HIT_sum"], cs["TCC_MISS_sum"]
            lines.append(f"L2 hit rate of `{nm}`: {h / max(h + m, 1):.3f} ({h:.4g} hits, {m:.4g} misses).")
        if cs.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) > 0:
            flops = cs["SQ_INSTS_VALU_MFMA_MOPS_F64"] * 512
            lines.append(f"FP64 matrix cores in `{nm}`: {flops / 1e9:.3g} GFLOP per dispatch (MOPS x 512), "
                         f"{flops / (ms[nm] * 1e-3) / 1e12:.2f} TFLOP/s = "
                         f"{flops / (ms[nm] * 1e-3) / 78.6e12:.1%} of the 78.6 TFLOP/s FP64 peak"
                         + (f"; SQ_VALU_MFMA_BUSY_CYCLES / (4 SIMDs x CUs x cycles) = "
                            f"{cs['SQ_VALU_MFMA_BUSY_CYCLES'] / (4 * CUS * CLOCK_HZ * ms[nm] * 1e-3):.1%}."
                            if "SQ_VALU_MFMA_BUSY_CYCLES" in cs else "."))
    with open(os.path.join(PROFILES, f"{out_name}.md"), "w") as f:
        f.write("\n".join(lines) + "\n")


def summarize_trace(trace_dir: str, workload: str, cmd: str, out_name: str) -> None:
    """Write profiles/<out_name>.md: the kernel statistics of a rocprofv3 --kernel-trace --stats run."""
    stats = _csv_rows(os.path.join(trace_dir, "**", "*kernel_stats.csv"))
    lines = [f"# Kernel trace: {WORKLOADS.get(workload, workload)}", "",
             "Command (from the repository root, on one MI355X):", "", "```", cmd, "```", "",
             "| kernel | calls | average us | share % |", "|---|---|---|---|"]
    for r in stats[:16]:
        lines.append(f"| `{_short(r['name'])[:80]}` | {r['calls']} | {float(r['averagens']) / 1e3:.1f} | "
                     f"{float(r['percentage']):.1f} |")
    with open(os.path.join(PROFILES, f"{out_name}.md"), "w") as f:
        f.write("\n".join(lines) + "\n")


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
    ap.add_argument("--summarize-pmc", nargs="+", metavar="ARG",
                    help="WORKLOAD NNZ K OUT_NAME DIR::COMMAND [DIR::COMMAND ...]: write profiles/OUT_NAME.md "
                         "(and the traffic / VALU json of the edge pass) from rocprofv3 --pmc CSV output and exit")
    ap.add_argument("--summarize-trace", nargs=4, metavar=("TRACE_DIR", "WORKLOAD", "COMMAND", "OUT_NAME"),
                    help="write profiles/OUT_NAME.md from a rocprofv3 --kernel-trace --stats CSV run and exit")
    args = ap.parse_args()
    if args.summarize_pmc:
        w, nnz, k, out_name, *runs = args.summarize_pmc
        summarize_pmc(w, int(nnz), int(k), out_name, runs)
        return 0
    if args.summarize_trace:
        d, w, cmd, out_name = args.summarize_trace
        summarize_trace(d, w, cmd, out_name)
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
        pspec_hvp call (edge pass + epilogue), the fixed-U Riemannian Hessian of the truncated-CG loop
        (pspec_rhess), the gather floor of the edge pass, one k-means step on U's rows (k clusters) with its
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
            # the truncated-CG call at a fixed U: G (the gradient at U) from the hvp call above
            "rhess": lambda: pspec.rhess(dg, U, V, G, p, eps, RH=RH, MG=MG, F_col=Fc),
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
            # row schedule of the graph handle; with ascending rows the objective pass visits each
            # undirected edge once
            "schedule": dg.info(),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": ("fused grad+HVP edge pass (light rows, heavy chunks, split-row combine; "
                       "at 9 <= k <= 16 the light rows also form the Gram products of the projection)"),
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
