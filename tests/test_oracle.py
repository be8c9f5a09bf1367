"""The FP64 oracle against its pins (CPU only)."""
import numpy as np
import pytest

import oracle as orc
from paper_2605_26975_amd import gen
from tests import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin, oracle_lib):
    pin(oracle_lib)


def test_oracle_threads_deterministic(oracle_lib):
    """Per-row work runs in parallel but sums are taken in row order: repeated calls agree bit for bit."""
    from paper_2605_26975_amd import gen

    g = gen.sbm_bernoulli(1000, 4, 0.05, 0.002)
    U = gen.block(g.n, 4, gen.SEED_U).astype(np.float64)
    V = gen.block(g.n, 4, gen.SEED_V).astype(np.float64)
    a = oracle_lib.hvp(g.rowptr, g.col, g.w, U, V, 1.3, 1e-8)
    b = oracle_lib.hvp(g.rowptr, g.col, g.w, U, V, 1.3, 1e-8)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_golden_worked_examples(oracle_lib):
    """Hand-worked cases stored in tests/golden/worked_examples.txt (derivations in the file)."""
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.txt")
    cases = 0
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, edges, u, p, F = [s.strip() for s in line.split("|")]
        p, F = float(p), float(F)
        U = np.array([float(x) for x in u.split()])[:, None]
        n = len(U)
        W = np.zeros((n, n))
        for e in edges.split(","):
            i, j, wv = e.split()
            W[int(i), int(j)] = W[int(j), int(i)] = float(wv)
        rp, c, w = pins.csr_from_dense(W)
        got, _, _, _ = oracle_lib.objective(rp, c, w, U, p)
        assert abs(got - F) <= 1e-15 * max(1.0, abs(F)), (name, got, F)
        cases += 1
    assert cases >= 4


def test_permuted_graph_is_the_same_graph(oracle_lib):
    """gen.permute relabels nodes only: degrees and weights move with the nodes, the CSR stays
    symmetric with ascending columns, and the oracle's outputs are the permuted originals."""
    g = gen.sbm_bernoulli(600, 3, 0.05, 0.004)
    h = gen.permute(g, seed=3)
    perm = np.random.default_rng(3).permutation(g.n)
    assert h.nnz == g.nnz
    assert np.array_equal(np.diff(h.rowptr)[perm], np.diff(g.rowptr))
    Wg, Wh = g.to_dense(), h.to_dense()
    assert np.array_equal(Wh[np.ix_(perm, perm)], Wg)
    for i in range(h.n):
        c = h.col[h.rowptr[i]:h.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0)
    U = gen.block(g.n, 4, gen.SEED_U).astype(np.float64)
    V = gen.block(g.n, 4, gen.SEED_V).astype(np.float64)
    Up, Vp = np.empty_like(U), np.empty_like(V)
    Up[perm], Vp[perm] = U, V
    HV, G, Fc = oracle_lib.hvp(g.rowptr, g.col, g.w.astype(np.float64), U, V, 1.3, 1e-8)
    HVp, Gp, Fcp = oracle_lib.hvp(h.rowptr, h.col, h.w.astype(np.float64), Up, Vp, 1.3, 1e-8)
    assert np.allclose(Fcp, Fc, rtol=1e-13)
    assert np.allclose(Gp[perm], G, rtol=1e-12, atol=1e-15)
    assert np.allclose(HVp[perm], HV, rtol=1e-12, atol=1e-15)


def test_delaunay_generator_is_a_triangulation():
    """gen.delaunay: symmetric, loop-free, unit weights, connected, and with exactly 3n - 3 - h
    undirected edges (Euler's formula for a triangulation of n points, h of them on the hull)."""
    from scipy.spatial import ConvexHull
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components

    n = 3000
    g = gen.delaunay(n, seed=5)
    h = len(ConvexHull(g.meta["points"]).vertices)
    assert g.nnz == 2 * (3 * n - 3 - h)
    assert np.all(g.w == 1.0)
    W = g.to_dense()
    assert np.array_equal(W, W.T) and np.all(np.diag(W) == 0)
    A = csr_matrix((g.w, g.col, g.rowptr), shape=(n, n))
    assert connected_components(A, directed=False)[0] == 1
    assert 5.9 < g.nnz / n < 6.0


def test_kmeans_step_pins():
    """orc.kmeans_step against facts that do not depend on it: rows placed on a centroid get that
    centroid at distance 0; in 1-D the nearest of sorted centroids is fixed by the midpoints between
    them (ties at a midpoint go to the lower index); member sums and counts add up to the column sums
    and n; per-cluster inertia obeys the parallel-axis identity sum ||x - c||^2 = sum ||x - m||^2 +
    n_j ||m - c||^2 about the cluster mean m; distances equal squared norms from numpy.linalg."""
    rng = np.random.default_rng(11)
    C = rng.normal(size=(5, 3))
    X = np.repeat(C, 4, axis=0)[rng.permutation(20)]
    lab, dist, stats = orc.kmeans_step(X, C)
    assert np.array_equal(C[lab], X) and np.all(dist == 0.0)
    assert np.array_equal(stats[:, 3], np.full(5, 4.0))
    # 1-D: midpoints
    c1 = np.array([[-1.0], [0.5], [2.0], [7.0]])
    x1 = np.concatenate([rng.uniform(-4, 10, 500), [-0.25, 1.25, 4.5]])[:, None]  # last three: exact ties
    lab1, _, _ = orc.kmeans_step(x1, c1)
    mids = (c1[1:, 0] + c1[:-1, 0]) / 2
    assert np.array_equal(lab1, np.searchsorted(mids, x1[:, 0], side="left"))
    # reordering the centroids relabels the rows the same way (away from the exact ties, whose
    # winner is the lower index and so depends on the order)
    perm = np.array([2, 0, 3, 1])
    lab1p, _, _ = orc.kmeans_step(x1, c1[perm])
    assert np.array_equal(perm[lab1p][:500], lab1[:500])
    # general data: conservation, parallel axis, brute-force distances
    X = rng.normal(size=(400, 6))
    C = rng.normal(size=(7, 6))
    lab, dist, stats = orc.kmeans_step(X, C)
    assert np.allclose(stats[:, :6].sum(axis=0), X.sum(axis=0), rtol=0, atol=1e-12)
    assert stats[:, 6].sum() == 400
    full = np.linalg.norm(X[:, None, :] - C[None, :, :], axis=2) ** 2
    assert np.array_equal(lab, np.argmin(full, axis=1))
    assert np.allclose(dist, full.min(axis=1), rtol=1e-14)
    for j in range(7):
        m = lab == j
        if m.sum() == 0:
            continue
        mean = X[m].mean(axis=0)
        pa = ((X[m] - mean) ** 2).sum() + m.sum() * ((mean - C[j]) ** 2).sum()
        assert abs(stats[j, 7] - pa) <= 1e-12 * pa


def test_lloyd_hand_example():
    """Two well separated pairs in 1-D, started from two points of the first pair: step 1 sends 0 to
    c0 = 0 and 1, 10, 11 to c1 = 1, moving c1 to 22/3; step 2 forms {0, 1} and {10, 11}, moving the
    centroids to 0.5 and 10.5; step 3 changes nothing.  Inertia 4 * 0.25 = 1."""
    X = np.array([[0.0], [1.0], [10.0], [11.0]])
    lab, C, inertia, steps = orc.lloyd(X, np.array([[0.0], [1.0]]))
    assert np.array_equal(lab, [0, 0, 1, 1])
    assert np.array_equal(C[:, 0], [0.5, 10.5])
    assert inertia == 1.0 and steps == 3



def test_induced_subgraph():
    """gen.induced keeps exactly the edges among kept nodes, renumbered in node order."""
    g = gen.sbm_bernoulli(500, 4, 0.03, 0.004)
    keep = np.random.default_rng(1).random(g.n) < 0.7
    h, ids = gen.induced(g, keep)
    assert np.array_equal(ids, np.flatnonzero(keep))
    assert np.array_equal(h.to_dense(), g.to_dense()[np.ix_(ids, ids)])
    for i in range(h.n):
        c = h.col[h.rowptr[i]:h.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0)
