"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by element.

Every entry of G and HV is held to |x_gpu - x_oracle| <= tau * S, S its forward-error scale from the
oracle (tests/gpu_util.py): tau = 4e-6 for the FP32 path, 1e-13 for the FP64 path.  F, and the
relative Frobenius error of G and HV over the block and over each column, must be below 1e-5
(FP32) or 1e-13 (FP64).
"""
import numpy as np
import pytest
import torch

from paper_2605_26975_amd import gen
from paper_2605_26975_amd import pspec
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module")
def sbm1000():
    return gen.sbm_bernoulli(1000, 4, 0.05, 0.002)


@pytest.mark.parametrize("p", [2.0, 1.6, 1.3, 1.1])
def test_sbm1000_fp64_plain_path(sbm1000, p):
    print(f"[case] sbm1000 f64 p={p}", flush=True)
    e = gu.compare(sbm1000, 4, p, 1e-8, torch.float64)
    gu.check(e, torch.float64)


@pytest.mark.parametrize("p", [2.0, 1.6, 1.3, 1.1])
def test_sbm1000_fp32_fused_path(sbm1000, p):
    print(f"[case] sbm1000 f32 p={p}", flush=True)
    e = gu.compare(sbm1000, 4, p, 1e-8, torch.float32)
    gu.check(e, torch.float32)


@pytest.mark.parametrize("k", [1, 3, 8, 13, 16, 32, 33])
@pytest.mark.parametrize("layout", ["separate", "interleaved"])
def test_multitile_ragged(k, layout):
    """50,000 nodes (195 full tiles and a ragged one), k from 1 to 33 (padded column lanes), U and V
    as separate arrays or as the two halves of one n x 2k array."""
    print(f"[case] sbm50k k={k} {layout}", flush=True)
    g = gen.sbm_edges(50_000, 16, 270_000, 30_000, 0.5, 1.5, seed=7)
    for dtype in (torch.float32, torch.float64):
        gu.check(gu.compare(g, k, 1.3, 1e-8, dtype, layout=layout), dtype)


def _hub_graph():
    """Light rows plus hubs of degree LIGHT_MAX (the light limit), LIGHT_MAX + 1 and 300 (one heavy
    chunk), CHUNK (exactly one chunk), CHUNK + 1 (two chunks) and 5000 (several chunks, combined
    afterwards)."""
    rng = np.random.default_rng(5)
    n = 6000
    i = [rng.integers(0, n, 30000)]
    j = [rng.integers(0, n, 30000)]
    L, C = pspec.LIGHT_MAX, pspec.CHUNK
    for hub, deg in ((0, 5000), (1, C + 1), (2, C), (3, 300), (4, L + 1), (5, L)):
        nb = rng.choice(np.arange(10, n), size=deg, replace=False)
        i.append(np.full(deg, hub))
        j.append(nb)
    i = np.concatenate(i)
    j = np.concatenate(j)
    g = gen.csr_from_edges(n, i, j, lambda lo, hi: gen.edge_uniform(3, lo, hi, 0.1, 1.0), name="hubs")
    return g


def expected_chunks(g, segs=8):
    """The schedule's chunk count, recomputed: one chunk per row of LIGHT_MAX + 1 .. CHUNK edges; a
    longer row is cut at the column-segment boundaries (bound[s] = first node j with
    rowptr[j] >= ceil(s nnz / segs)) and every piece into chunks of at most CHUNK edges."""
    L, C = pspec.LIGHT_MAX, pspec.CHUNK
    deg = g.degrees()
    bounds = [int(np.searchsorted(g.rowptr, (g.nnz * s + segs - 1) // segs, side="left")) for s in range(1, segs)]
    total = int(np.sum((deg > L) & (deg <= C)))
    for i in np.flatnonzero(deg > C):
        cols = g.col[g.rowptr[i]:g.rowptr[i + 1]]
        pos = [0] + [int(np.searchsorted(cols, b, side="left")) for b in bounds] + [len(cols)]
        total += sum((pos[s + 1] - pos[s] + C - 1) // C for s in range(segs))
    return total


@pytest.mark.parametrize("k", [4, 5, 32])
def test_heavy_and_split_rows(k):
    """Rows at and around LIGHT_MAX and CHUNK (light, single-chunk and split rows); k = 4 takes the
    4-lane row groups, whose light rows of up to 32 edges span up to 8 chunks of 4."""
    print(f"[case] hubs k={k}", flush=True)
    g = _hub_graph()
    dg = gu.device_graph(g, k)
    info = dg.info()
    deg = g.degrees()
    assert info["heavy_rows"] == int(np.sum(deg > pspec.LIGHT_MAX))
    assert info["split_rows"] == int(np.sum(deg > pspec.CHUNK))
    assert info["chunks"] == expected_chunks(g)
    assert info["split_rows"] >= 2 and info["heavy_rows"] >= 5
    for dtype in (torch.float64, torch.float32):
        gu.check(gu.compare(g, k, 1.2, 1e-8, dtype, dg=dg), dtype)


@pytest.mark.parametrize("layout", ["separate", "interleaved"])
def test_rmat_scale14_p105(layout):
    """Skewed degrees (R-MAT), k = 32, p = 1.05, eps = 1e-8; the light tiles in degree order."""
    print(f"[case] rmat14 {layout}", flush=True)
    g = gen.rmat(14, 16, 0.57, 0.19, 0.19, 0.1, 1.0, seed=9)
    dg = gu.device_graph(g, 32)
    assert dg.info()["degree_order"]
    gu.check(gu.compare(g, 32, 1.05, 1e-8, torch.float32, dg=dg, layout=layout), torch.float32)
    gu.check(gu.compare(g, 32, 1.05, 1e-8, torch.float64, dg=dg), torch.float64)


@pytest.mark.parametrize("k", [16, 32])
def test_degree_order_ragged_last_tile(k):
    """Degree order with a ragged last tile (n = 16,284, not a multiple of 256): the fused grad+HVP
    and the edge-once objective against the oracle, every entry within its bound."""
    print(f"[case] degree order ragged k={k}", flush=True)
    full = gen.rmat(14, 16, 0.57, 0.19, 0.19, 0.1, 1.0, seed=9)
    keep = np.ones(full.n, dtype=bool)
    keep[-100:] = False
    g, _ = gen.induced(full, keep, "rmat14-ragged")
    assert g.n % 256 != 0
    dg = gu.device_graph(g, k)
    info = dg.info()
    assert info["degree_order"] and info["ascending"] and info["split_rows"] > 0
    gu.check(gu.compare(g, k, 1.05, 1e-8, torch.float32, dg=dg, layout="interleaved"), torch.float32)
    gu.check(gu.compare(g, k, 1.05, 1e-8, torch.float64, dg=dg), torch.float64)


@pytest.mark.parametrize("k", [3, 4, 8, 16, 32])
def test_gather_floor_visits_every_edge_once(k):
    """The gather-floor reference pass (the edge kernels with the arithmetic replaced by plain sums)
    adds each visited entry's weight into the row's first output, so that output must equal the row
    sums of w in every column: every stored entry visited exactly once by the light groups (4-, 8-
    and 16-lane), the heavy chunks and the split-row combine, on the hub graph (light, single-chunk
    and split rows) and on R-MAT-14 (degree-ordered tiles)."""
    for g in (_hub_graph(), gen.rmat(14, 16, 0.57, 0.19, 0.19, 0.1, 1.0, seed=9)):
        print(f"[case] gather floor {g.name} k={k}", flush=True)
        dg = gu.device_graph(g, k)
        U, V = gu.inputs(g.n, k)
        _, G = pspec.hvp_gather_floor(dg, torch.as_tensor(U).cuda(), torch.as_tensor(V).cuda())
        torch.cuda.synchronize()
        w = g.w.astype(np.float64)
        rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
        want = np.bincount(rows, weights=w, minlength=g.n)
        got = G.double().cpu().numpy()
        # FP32 sums of at most a few thousand positive terms in some order
        bound = 1e-6 * np.bincount(rows, weights=np.abs(w), minlength=g.n)[:, None] * np.log2(2 + np.diff(g.rowptr))[:, None]
        err = np.abs(got - want[:, None])
        assert np.all(err <= bound + 1e-30), (g.name, k, float(np.max(err - bound)))
        dg.close()


def test_fp64_degree_order_on_uniform_graph():
    """Near-uniform degrees (SBM, n = 3,000, a ragged last tile): FP32 calls keep node order, FP64
    calls take degree order, both from the same handle; grad+HVP, objective and the Riemannian call
    against the oracle, every entry within its bound."""
    print("[case] fp64 degree order sbm3000", flush=True)
    g = gen.sbm_bernoulli(3000, 3, 0.01, 0.001, seed=21)
    assert g.n % 256 != 0
    d = g.degrees()
    assert d.max() <= pspec.LIGHT_MAX and d.std() < d.mean()
    dg = gu.device_graph(g, 16)
    assert not dg.info()["degree_order"]
    for dtype in (torch.float64, torch.float32):
        gu.check(gu.compare(g, 16, 1.1, 1e-8, dtype, dg=dg), dtype)


def test_degree_order_rule():
    """FP32 calls take the light tiles in degree order exactly when the degrees of the light rows
    (at most LIGHT_MAX entries) have a coefficient of variation above 1, recomputed here in NumPy
    (FP64 calls take degree order on every graph)."""
    graphs = [gen.sbm_bernoulli(1000, 4, 0.05, 0.002), gen.rmat(14, 16, 0.57, 0.19, 0.19, 0.1, 1.0, seed=9),
              gen.rmat(12, 8, 0.57, 0.19, 0.19, 0.1, 1.0, seed=3), _hub_graph(), gen.grid3d(16),
              gen.knn_mixture(5_000, 4, 10, 1.0, 20.0, seed=4)]
    seen = set()
    for g in graphs:
        d = g.degrees()
        light = d[d <= pspec.LIGHT_MAX].astype(np.float64)
        want = bool(light.mean() > 0 and light.var() > light.mean() ** 2)
        got = gu.device_graph(g, 4).info()["degree_order"]
        print(f"{g.name}: cv {light.std() / light.mean():.2f} degree order {got}", flush=True)
        assert got == want
        seen.add(got)
    assert seen == {True, False}


def test_knn_graph_p13():
    print("[case] knn20k", flush=True)
    g = gen.knn_mixture(20_000, 8, 10, 1.0, 20.0, seed=4)
    gu.check(gu.compare(g, 8, 1.3, 1e-8, torch.float32), torch.float32)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_empty_graph_and_single_node(dtype):
    print(f"[case] empty {dtype}", flush=True)
    for n in (1, 300):
        g = gen.Graph(n=n, rowptr=np.zeros(n + 1, np.int64), col=np.zeros(0, np.int32), w=np.zeros(0, np.float32))
        U, V = gu.inputs(n, 4)
        dg = gu.device_graph(g, 4)
        HV, G, Fc = gu.gpu_hvp(dg, U, V, 1.5, 1e-8, dtype)
        assert np.all(Fc == 0.0) and np.all(G == 0.0) and np.all(HV == 0.0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_disconnected_indicators_are_exact_zeros(dtype):
    """Per-component constant columns: every x = 0, so F = 0 and G = 0 exactly (a zero-difference
    edge must contribute exactly nothing)."""
    print(f"[case] indicators {dtype}", flush=True)
    g = gen.sbm_bernoulli(400, 2, 0.1, 0.0, seed=3)
    U = np.zeros((400, 3), np.float32)
    U[:200, 0] = 1.0
    U[200:, 1] = 1.0
    U[:200, 2] = 2.0
    U[200:, 2] = -0.5
    V = gen.block(400, 3, 2)
    dg = gu.device_graph(g, 3)
    for p in (2.0, 1.5, 1.05):
        HV, G, Fc = gu.gpu_hvp(dg, U, V, p, 1e-8, dtype)
        assert np.all(Fc == 0.0) and np.all(G == 0.0)
        HVo, _, _ = gu.oracle_hvp(g, U, V, p, 1e-8)
        _, SH = gu.oracle_scales(g, U, V, p, 1e-8)
        assert gu.ew(HV, HVo, SH) <= gu.TOLS[dtype]["tau"]


def test_zero_column_is_nan():
    g = gen.sbm_bernoulli(300, 2, 0.1, 0.01, seed=3)
    U, V = gu.inputs(300, 3)
    U[:, 1] = 0.0
    HV, G, Fc = gu.gpu_hvp(gu.device_graph(g, 3), U, V, 1.5, 1e-8, torch.float32)
    assert np.isnan(Fc[1]) and np.all(np.isnan(G[:, 1])) and np.all(np.isnan(HV[:, 1]))
    assert np.all(np.isfinite(G[:, [0, 2]])) and np.all(np.isfinite(HV[:, [0, 2]]))


def test_interleaved_and_padded_layouts_match():
    """U and V as the two halves of one n x 2k array, and blocks with ld > k, give bit-identical
    results to the plain layout (same arithmetic in the same order)."""
    g = gen.sbm_edges(20_000, 8, 100_000, 10_000, 0.5, 1.5, seed=11)
    k = 16
    U, V = gu.inputs(g.n, k)
    dg = gu.device_graph(g, k)
    Ut = torch.as_tensor(U).cuda()
    Vt = torch.as_tensor(V).cuda()
    HV0, G0, F0 = pspec.hvp(dg, Ut, Vt, 1.1, 1e-8)
    P = torch.cat([Ut, Vt], dim=1).contiguous()
    HV1, G1, F1 = pspec.hvp(dg, P[:, :k], P[:, k:], 1.1, 1e-8)
    big = torch.zeros((g.n, 24), dtype=torch.float32, device="cuda")
    big[:, :k] = Ut
    bigV = torch.zeros((g.n, 20), dtype=torch.float32, device="cuda")
    bigV[:, :k] = Vt
    HVo = torch.zeros((g.n, 40), dtype=torch.float32, device="cuda")
    Go = torch.zeros((g.n, 17), dtype=torch.float32, device="cuda")
    HV2, G2, F2 = pspec.hvp(dg, big[:, :k], bigV[:, :k], 1.1, 1e-8, HV=HVo[:, 3:3 + k], G=Go[:, :k])
    torch.cuda.synchronize()
    for a, b in ((HV0, HV1), (G0, G1), (F0, F1), (HV0, HV2), (G0, G2), (F0, F2)):
        assert torch.equal(a, b)
    assert torch.all(HVo[:, :3] == 0) and torch.all(HVo[:, 3 + k:] == 0) and torch.all(Go[:, k:] == 0)


def test_deterministic():
    g = gen.rmat(13, 16, 0.57, 0.19, 0.19, 0.1, 1.0, seed=2)
    U, V = gu.inputs(g.n, 8)
    dg = gu.device_graph(g, 8)
    a = gu.gpu_hvp(dg, U, V, 1.2, 1e-8, torch.float32)
    b = gu.gpu_hvp(dg, U, V, 1.2, 1e-8, torch.float32)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_objective_and_grad_entry_points_agree_with_hvp():
    """grad and hvp form the same G and F_col bit for bit.  The objective visits each undirected edge
    once when the rows' columns ascend (equal to rounding); with the rows shuffled it visits every
    stored entry, like the other calls, and agrees bit for bit."""
    g = gen.sbm_edges(30_000, 8, 150_000, 15_000, 0.5, 1.5, seed=12)
    k = 8
    U, V = gu.inputs(g.n, k)
    Ut, Vt = torch.as_tensor(U).cuda(), torch.as_tensor(V).cuda()
    for gg, ascending in ((g, True), (gu.shuffled(g), False)):
        dg = gu.device_graph(gg, k)
        assert dg.info()["ascending"] == ascending
        HV, G, Fc = pspec.hvp(dg, Ut, Vt, 1.4, 1e-8)
        G2, Fc2 = pspec.grad(dg, Ut, 1.4)
        F3, Fc3 = pspec.objective(dg, Ut, 1.4)
        torch.cuda.synchronize()
        assert torch.equal(G, G2) and torch.equal(Fc, Fc2)
        if ascending:  # FP32 row sums over different entry sets
            assert float(((Fc3 - Fc) / Fc).abs().max()) <= gu.TOLS[torch.float32]["F"]
        else:
            assert torch.equal(Fc, Fc3)
        assert float(F3) == pytest.approx(float(Fc3.sum()), rel=1e-15)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("k", [4, 16, 32])
def test_objective_edge_once_vs_oracle(dtype, k):
    """The objective over ascending rows (entries j > i of light rows, of single-chunk heavy rows and
    of every column segment of split rows, chunks that hold none skipped) against the oracle's
    1/2 sum over every stored entry, and the same graph with shuffled rows (every entry visited)."""
    print(f"[case] objective edge-once rmat14 k={k} {dtype}", flush=True)
    g = gen.rmat(14, 16, 0.57, 0.19, 0.19, 0.1, 1.0, seed=9)
    U, _ = gu.inputs(g.n, k)
    _, _, Fco = gu.oracle_hvp(g, U, U, 1.05, 1e-8)
    tol = gu.TOLS[dtype]["F"]
    for gg, ascending in ((g, True), (gu.shuffled(g, seed=7), False)):
        dg = gu.device_graph(gg, k)
        info = dg.info()
        assert info["ascending"] == ascending and info["split_rows"] > 0
        Fg, Fcg = gu.gpu_objective(dg, U, 1.05, dtype)
        err = float(np.max(np.abs(Fcg - Fco) / np.abs(Fco)))
        print(f"ascending={ascending} Fcol err {err:.2e}", flush=True)
        assert err <= tol
        assert abs(Fg - Fco.sum()) <= tol * abs(Fco.sum())


def test_objective_edge_once_with_loops_duplicates_and_one_descent():
    """Self-loops (column i in row i: not above i, and x = 0 anyway) and duplicate entries keep the
    rows ascending and the objective equal to the oracle's; one descending pair inside a long row
    turns the edge-once pass off for the whole graph."""
    base = gen.rmat(12, 8, 0.57, 0.19, 0.19, 0.1, 1.0, seed=3)
    n = base.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(base.rowptr))
    i = np.concatenate([rows, np.arange(0, n, 7, dtype=np.int64)])
    j = np.concatenate([base.col.astype(np.int64), np.arange(0, n, 7, dtype=np.int64)])
    w = np.concatenate([base.w, np.full((n + 6) // 7, 0.5, dtype=np.float32)])
    dup = (i % 5 == 0) & (j > i)  # duplicate both directions of some edges
    i, j, w = (np.concatenate([i, i[dup], j[dup]]), np.concatenate([j, j[dup], i[dup]]),
               np.concatenate([w, w[dup], w[dup]]))
    order = np.lexsort((j, i))
    i, j, w = i[order], j[order], w[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, i + 1, 1)
    g = gen.Graph(n, np.cumsum(rowptr), j.astype(np.int32), w.astype(np.float32), name="loops-dups")
    k = 8
    U, _ = gu.inputs(n, k)
    _, _, Fco = gu.oracle_hvp(g, U, U, 1.3, 1e-8)
    dg = gu.device_graph(g, k)
    assert dg.info()["ascending"]
    _, Fcg = gu.gpu_objective(dg, U, 1.3, torch.float64)
    assert np.max(np.abs(Fcg - Fco) / np.abs(Fco)) <= 1e-13
    # swap two entries of the longest row: still a valid graph, no longer ascending
    r = int(np.argmax(np.diff(g.rowptr)))
    col2, w2 = g.col.copy(), g.w.copy()
    a, b = g.rowptr[r], g.rowptr[r + 1] - 1
    col2[[a, b]], w2[[a, b]] = col2[[b, a]], w2[[b, a]]
    g2 = gen.Graph(n, g.rowptr, col2, w2, name="one-descent")
    dg2 = gu.device_graph(g2, k)
    assert not dg2.info()["ascending"]
    _, Fcg2 = gu.gpu_objective(dg2, U, 1.3, torch.float64)
    assert np.max(np.abs(Fcg2 - Fco) / np.abs(Fco)) <= 1e-13


def test_invalid_csr_and_arguments_are_rejected():
    n = 100
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    rowptr[1:] = 2
    rowptr[-1] = 2
    col = torch.tensor([5, 100], dtype=torch.int32, device="cuda")  # 100 is out of range
    w = torch.ones(2, dtype=torch.float32, device="cuda")
    rowptr[1:] = 2
    with pytest.raises(pspec.PSpecError) as ei:
        pspec.Graph(rowptr, col, w, 4)
    assert ei.value.status == 1
    bad_rp = torch.tensor([0, 3, 2] + [2] * (n - 2), dtype=torch.int64, device="cuda")
    with pytest.raises(pspec.PSpecError):
        pspec.Graph(bad_rp, torch.tensor([1, 2], dtype=torch.int32, device="cuda"), w, 4)
    g = gen.sbm_bernoulli(200, 2, 0.1, 0.01)
    dg = gu.device_graph(g, 4)
    U = torch.randn(200, 4, device="cuda")
    for p in (1.0, 2.5, float("nan")):
        with pytest.raises(pspec.PSpecError):
            pspec.objective(dg, U, p)
    with pytest.raises(pspec.PSpecError):
        pspec.hvp(dg, U, U, 1.5, 0.0)
    with pytest.raises(pspec.PSpecError):
        pspec.objective(dg, torch.randn(200, 5, device="cuda"), 1.5)  # k > k_max
    with pytest.raises(pspec.PSpecError):
        pspec.hvp(dg, U, U, 1.5, 1e-8, HV=U)  # output overlaps input
    dg64 = pspec.Graph.from_host(g, "cuda", k_max=4, weight_dtype=torch.float64)
    with pytest.raises(pspec.PSpecError) as ei:
        pspec.objective(dg64, U, 1.5)  # FP32 arithmetic with FP64 weights
    assert ei.value.status == 2
    F, _ = pspec.objective(dg64, U.double(), 1.5)
    assert torch.isfinite(F)


def test_size_limits_are_rejected_before_any_launch():
    """The documented limits: a block spanning 4 GiB or more (32-bit buffer offsets) and k_max above
    PSPEC_K_MAX return PSPEC_ERR_UNSUPPORTED from the host checks.  The oversized blocks are real
    small tensors given a leading dimension that makes their extent exceed 4 GiB, so nothing may be
    launched on them; the calls are made through the C ABI to bypass the binding's own shape checks."""
    import ctypes

    g = gen.sbm_bernoulli(200, 2, 0.1, 0.01)
    dg = gu.device_graph(g, 4)
    lib = pspec.lib()
    stream = torch.cuda.current_stream().cuda_stream
    for dt, dtype in ((0, torch.float32), (1, torch.float64)):
        es = 4 if dt == 0 else 8
        big = (1 << 32) // (es * (g.n - 1)) + 1  # (n - 1) * big * es >= 4 GiB
        U = torch.randn(g.n, 4, dtype=dtype, device="cuda")
        V = torch.randn(g.n, 4, dtype=dtype, device="cuda")
        HV, G = torch.empty_like(U), torch.empty_like(U)
        Fc = torch.empty(4, dtype=torch.float64, device="cuda")
        HV0 = HV.clone()
        for ldu, ldv in ((big, 4), (4, big)):
            st = lib.pspec_hvp(dg.handle, dt, 4, U.data_ptr(), ldu, V.data_ptr(), ldv, 1.5, 1e-8, HV.data_ptr(), 4,
                               G.data_ptr(), 4, Fc.data_ptr(), ctypes.c_void_p(stream))
            assert st == 2, (dt, ldu, ldv, st)
            assert b"4 GiB" in lib.pspec_last_error()
        torch.cuda.synchronize()
        assert torch.equal(HV, HV0)  # nothing was written
    with pytest.raises(pspec.PSpecError) as ei:
        gu.device_graph(g, pspec.K_MAX + 1)
    assert ei.value.status in (1, 2)
    dg.close()


# --- Grassmann steps --------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("k", [1, 4, 13, 32, 64])
def test_project_and_retract_vs_oracle(dtype, k):
    import oracle as orc

    print(f"[case] dense {dtype} k={k}", flush=True)
    rng = np.random.default_rng(k)
    n = 5000 + k
    U64, _ = np.linalg.qr(rng.standard_normal((n, k)))
    Z64 = rng.standard_normal((n, k))
    X64 = rng.standard_normal((n, k))
    U = torch.as_tensor(U64).to(dtype).cuda()
    Z = torch.as_tensor(Z64).to(dtype).cuda()
    X = torch.as_tensor(X64).to(dtype).cuda()
    Uh = U.double().cpu().numpy()
    Zh = Z.double().cpu().numpy()
    Xh = X.double().cpu().numpy()
    # element-wise scales: |Z| + |U| |M| (+ |X| |MX|) for the projection, |U|^T |Z| for M,
    # |Y| |R^-1| for the retraction; FP64 arithmetic inside, so the FP32 outputs' rounding dominates
    tol = 1e-6 if dtype == torch.float32 else 1e-13
    tau = 1e-6 if dtype == torch.float32 else 1e-12
    out, M = pspec.project(U, Z)
    ref, Mref = orc.project(Uh, Zh)
    assert gu.rel(M.cpu().numpy(), Mref) < 1e-12
    assert gu.ew(M.cpu().numpy(), Mref, np.abs(Uh).T @ np.abs(Zh)) <= 1e-12
    assert gu.rel(out.double().cpu().numpy(), ref) < tol
    assert gu.ew(out.double().cpu().numpy(), ref, np.abs(Zh) + np.abs(Uh) @ np.abs(Mref)) <= tau
    MX = torch.as_tensor(rng.standard_normal((k, k))).cuda()
    out2, _ = pspec.project(U, Z, X=X, MX=MX)
    MXh = MX.cpu().numpy()
    ref2 = ref - Xh @ MXh
    assert gu.rel(out2.double().cpu().numpy(), ref2) < tol
    assert gu.ew(out2.double().cpu().numpy(), ref2,
                 np.abs(Zh) + np.abs(Uh) @ np.abs(Mref) + np.abs(Xh) @ np.abs(MXh)) <= tau
    Zc = Z.clone()
    pspec.project(U, Zc, out=Zc)  # in place
    assert torch.equal(Zc, out)
    eta = out
    for t in (0.0, 0.3, 2.0):
        Q, R = pspec.retract(U, eta, t)
        Qref = orc.retract(Uh, eta.double().cpu().numpy(), t)
        Qh = Q.double().cpu().numpy()
        assert gu.rel(Qh, Qref) < (3e-6 if dtype == torch.float32 else 1e-12), t
        Y = Uh + t * eta.double().cpu().numpy()
        SQ = np.abs(Y) @ np.abs(np.linalg.inv(Qref.T @ Y))
        assert gu.ew(Qh, Qref, SQ) <= (1e-6 if dtype == torch.float32 else 1e-10), t
        assert np.max(np.abs(Qh.T @ Qh - np.eye(k))) < (1e-5 if dtype == torch.float32 else 1e-12)
        Rh = R.cpu().numpy()
        assert np.all(np.diag(Rh) > 0) and np.all(np.tril(Rh, -1) == 0)
    d = pspec.dot(Z, X)
    assert float(d) == pytest.approx(float(np.sum(Zh * Xh)), rel=1e-12)
    Y = Z.clone()
    pspec.axpby(0.5, X, -2.0, Y)
    assert gu.rel(Y.double().cpu().numpy(), 0.5 * Xh - 2.0 * Zh) < (1e-7 if dtype == torch.float32 else 1e-15)
    assert gu.ew(Y.double().cpu().numpy(), 0.5 * Xh - 2.0 * Zh, 0.5 * np.abs(Xh) + 2.0 * np.abs(Zh)) <= (
        2 ** -23 if dtype == torch.float32 else 2 ** -52)
    Uc = U.clone()
    pspec.retract(Uc, eta, 0.3, out=Uc)  # in place
    assert gu.rel(Uc.double().cpu().numpy(), orc.retract(Uh, eta.double().cpu().numpy(), 0.3)) < (
        3e-6 if dtype == torch.float32 else 1e-12)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_dense_strided_layouts_are_bit_identical(dtype):
    """The dense kernels move rows as 16-byte vectors when every leading dimension allows it and
    element by element otherwise; both visit the rows and columns in the same order, so contiguous
    blocks, column slices of a 2k-wide buffer (vector path) and slices with ld = k + 1 (element
    path) give identical bits."""
    k, n = 16, 3001
    print(f"[case] dense strided {dtype}", flush=True)
    rng = np.random.default_rng(7)
    U64, _ = np.linalg.qr(rng.standard_normal((n, k)))
    blocks = {nm: torch.as_tensor(a).to(dtype).cuda() for nm, a in
              (("U", U64), ("Z", rng.standard_normal((n, k))), ("X", rng.standard_normal((n, k))))}
    MX = torch.as_tensor(rng.standard_normal((k, k))).cuda()

    def laid_out(width):
        out = {}
        for nm, a in blocks.items():
            buf = torch.full((n, width), float("nan"), dtype=dtype, device="cuda")
            buf[:, :k] = a
            out[nm] = buf[:, :k]
        return out

    def run(b):
        P, M = pspec.project(b["U"], b["Z"], X=b["X"], MX=MX)
        Q, R = pspec.retract(b["U"], b["Z"], 0.7)
        d = pspec.dot(b["Z"], b["X"])
        Y = b["Z"].clone()
        pspec.axpby(0.5, b["X"], -2.0, Y)
        return [P, M, Q, R, d, Y]

    ref = run(blocks)
    for width in (2 * k, k + 1):
        got = run(laid_out(width))
        for a, b in zip(ref, got):
            assert torch.equal(a, b), width


@pytest.mark.parametrize("k", [16, 32])
def test_modes_agree_bitwise_with_heavy_rows(k):
    """With light, heavy single-chunk and split rows, every entry point partitions the rows and
    chunks the same way, so the per-column objective agrees bit for bit across grad, hvp and rhvp,
    and grad's G equals hvp's G.  The objective agrees with them bit for bit when it visits every
    stored entry (shuffled rows) and to FP32 rounding when it visits each undirected edge once."""
    print(f"[case] modes agree rmat14 k={k}", flush=True)
    g = gen.rmat(14, 16, 0.57, 0.19, 0.19, 0.1, 1.0, seed=9)
    U, V = gu.inputs(g.n, k)
    Ut, Vt = torch.as_tensor(U).cuda(), torch.as_tensor(V).cuda()
    p, eps = 1.05, 1e-8
    for gg, ascending in ((g, True), (gu.shuffled(g), False)):
        dg = gu.device_graph(gg, k)
        info = dg.info()
        assert info["heavy_rows"] > 0 and info["split_rows"] > 0 and info["ascending"] == ascending
        HV, G, Fc = pspec.hvp(dg, Ut, Vt, p, eps)
        G2, Fc2 = pspec.grad(dg, Ut, p)
        F3, Fc3 = pspec.objective(dg, Ut, p)
        RH, RG, MG, Fc4 = pspec.rhvp(dg, Ut, Vt, p, eps)
        torch.cuda.synchronize()
        assert torch.equal(G, G2)
        for other in (Fc2, Fc4):
            assert torch.equal(Fc, other)
        if ascending:  # FP32 row sums over different entry sets
            assert float(((Fc3 - Fc) / Fc).abs().max()) <= gu.TOLS[torch.float32]["F"]
        else:
            assert torch.equal(Fc, Fc3)


def test_dense_calls_on_two_streams_do_not_share_a_workspace():
    """The binding keeps one dense workspace per stream: projections issued on two streams at once
    give the same bits as on one stream."""
    print("[case] project on two streams", flush=True)
    n, k = 300_000, 8
    U = torch.as_tensor(gen.block(n, k, gen.SEED_U)).cuda()
    Z1 = torch.as_tensor(gen.block(n, k, gen.SEED_V)).cuda()
    Z2 = torch.as_tensor(gen.block(n, k, 11)).cuda()
    ref1 = pspec.project(U, Z1)[0].clone()
    ref2 = pspec.project(U, Z2)[0].clone()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    outs = []
    for _ in range(4):
        with torch.cuda.stream(s1):
            o1 = pspec.project(U, Z1)[0]
        with torch.cuda.stream(s2):
            o2 = pspec.project(U, Z2)[0]
        outs.append((o1, o2))
    torch.cuda.synchronize()
    for o1, o2 in outs:
        assert torch.equal(o1, ref1) and torch.equal(o2, ref2)
