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


def _dense_scales(W, U, V, p, eps):
    """The error scales of oracle_error_scales from their definition, over a dense weight matrix."""
    n, k = U.shape
    q = abs(p - 2.0)
    phi = lambda x: np.sign(x) * np.abs(x) ** (p - 1.0)  # noqa: E731
    psi = lambda x: np.maximum(np.abs(x), eps) ** (p - 2.0)  # noqa: E731
    kap = lambda x: 1.0 + q * np.abs(np.log2(np.abs(x)))  # noqa: E731
    kape = lambda x: 1.0 + q * np.abs(np.log2(np.maximum(np.abs(x), eps)))  # noqa: E731
    SG = np.zeros((n, k))
    SH = np.zeros((n, k))
    for l in range(k):
        u, v = U[:, l], V[:, l]
        D = np.sum(np.abs(u) ** p)
        F = 0.5 * sum(W[i, j] * abs(u[i] - u[j]) ** p for i in range(n) for j in range(n)) / D
        L = np.array([sum(W[i, j] * phi(u[i] - u[j]) for j in range(n)) for i in range(n)])
        g = (p / D) * (L - F * phi(u))
        for i in range(n):
            s = sum(W[i, j] * abs(phi(u[i] - u[j])) * kap(u[i] - u[j]) for j in range(n) if u[i] != u[j])
            SG[i, l] = (p / D) * (s + F * abs(phi(u[i])) * (kap(u[i]) if u[i] != 0 else 0.0))
        a = float(np.dot(phi(u), v))
        A = sum(abs(phi(u[i]) * v[i]) * kap(u[i]) for i in range(n) if u[i] != 0)
        B = float(np.sum(SG[:, l] * np.abs(v)))
        for i in range(n):
            s = sum(W[i, j] * psi(u[i] - u[j]) * abs(v[i] - v[j]) * kape(u[i] - u[j]) for j in range(n))
            SH[i, l] = (p / D) * ((p - 1.0) * s + F * (p - 1.0) * psi(u[i]) * abs(v[i]) * kape(u[i])
                                  + SG[i, l] * abs(a) + abs(g[i]) * A + abs(phi(u[i])) * B)
    return SG, SH


@pytest.mark.parametrize("p", [2.0, 1.3, 1.05])
def test_error_scales(oracle_lib, p):
    """The parity tolerances' per-entry scales: equal to their definition on a dense 9-node graph
    (with an exact tie, a zero entry and a sub-eps difference); never below |G| or |HV|; at p = 2
    they reduce to (2/D)(sum_j w |u_i - u_j| + F |u_i|) for the gradient."""
    rng = np.random.default_rng(11)
    W = pins.random_sym_weights(9, 0.6, rng)
    U = rng.normal(size=(9, 3))
    U[2, 0] = U[5, 0]            # exact tie on an edge or not: x = 0
    U[4, 1] = 0.0                # phi_p(0) = 0
    U[7, 2] = U[1, 2] + 3e-9     # |x| below eps
    V = rng.normal(size=(9, 3))
    rowptr, col, w = pins.csr_from_dense(W)
    SG, SH = oracle_lib.error_scales(rowptr, col, w, U, V, p, 1e-8)
    SGd, SHd = _dense_scales(W, U, V, p, 1e-8)
    assert np.allclose(SG, SGd, rtol=1e-12, atol=0) and np.allclose(SH, SHd, rtol=1e-12, atol=0)
    HV, G, _ = oracle_lib.hvp(rowptr, col, w, U, V, p, 1e-8)
    assert np.all(SG >= np.abs(G)) and np.all(SH >= np.abs(HV))
    if p == 2.0:
        D = np.sum(U ** 2, axis=0)
        F = np.array([0.5 * np.sum(W * (U[:, l][:, None] - U[:, l][None, :]) ** 2) / D[l] for l in range(3)])
        absx = np.abs(U[:, None, :] - U[None, :, :])
        ref = (2.0 / D) * (np.einsum("ij,ijl->il", W, absx) + F * np.abs(U))
        assert np.allclose(SG, ref, rtol=1e-12, atol=0)
    # larger graph: the bounds hold everywhere
    g = gen.sbm_bernoulli(300, 3, 0.1, 0.01, seed=3)
    U = gen.block(g.n, 4, gen.SEED_U).astype(np.float64)
    V = gen.block(g.n, 4, gen.SEED_V).astype(np.float64)
    SG, SH, SHs = oracle_lib.error_scales(g.rowptr, g.col, g.w, U, V, p, 1e-8, sparse=True)
    HV, G, _ = oracle_lib.hvp(g.rowptr, g.col, g.w, U, V, p, 1e-8)
    HVs = oracle_lib.hvp_sparse(g.rowptr, g.col, g.w, U, V, p, 1e-8)
    assert np.all(SG >= np.abs(G)) and np.all(SH >= np.abs(HV))
    assert np.all(SHs >= np.abs(HVs)) and np.all(SHs <= SH)
