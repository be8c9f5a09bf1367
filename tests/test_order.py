"""CPU: the library's reverse Cuthill-McKee relabelling (pspec_rcm_order, host code) and
gen.relabel.  RCM is pinned by what it must achieve on graphs whose best bandwidth is known (a
path: 1; a w x h grid: about min(w, h)), by scipy's implementation of the same method as a quality
reference, and by the permutation property; gen.relabel by the dense adjacency it produces."""
import numpy as np
import pytest

from paper_2605_26975_amd import gen, pspec


def _bandwidth(g, perm):
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    return int(np.abs(perm[rows] - perm[g.col.astype(np.int64)]).max()) if g.nnz else 0


def _shuffled(g, seed):
    return gen.relabel(g, np.random.default_rng(seed).permutation(g.n))


def _grid2d(w, h):
    idx = np.arange(w * h).reshape(h, w)
    i = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    j = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return gen.csr_from_edges(w * h, i, j, lambda lo, hi: np.ones(len(lo), dtype=np.float32), name="grid2d")


def test_rcm_is_a_permutation_and_deterministic():
    for g in (gen.sbm_bernoulli(600, 3, 0.05, 0.004), gen.delaunay(3000, seed=2)):
        p1 = pspec.rcm_order(g.rowptr, g.col)
        assert np.array_equal(np.sort(p1), np.arange(g.n))
        assert np.array_equal(p1, pspec.rcm_order(g.rowptr, g.col))


def test_rcm_path_and_grid_bandwidth():
    n = 500
    path = gen.csr_from_edges(n, np.arange(n - 1), np.arange(1, n),
                              lambda lo, hi: np.ones(len(lo), dtype=np.float32))
    g = _shuffled(path, 1)
    assert _bandwidth(g, np.arange(n)) > 100
    assert _bandwidth(g, pspec.rcm_order(g.rowptr, g.col)) == 1
    grid = _shuffled(_grid2d(40, 25), 2)
    bw = _bandwidth(grid, pspec.rcm_order(grid.rowptr, grid.col))
    assert bw <= 26, bw


def test_rcm_matches_scipy_quality_on_delaunay():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import reverse_cuthill_mckee

    g = gen.delaunay(1 << 14, seed=6)
    ours = _bandwidth(g, pspec.rcm_order(g.rowptr, g.col))
    A = csr_matrix((np.ones(g.nnz), g.col, g.rowptr), shape=(g.n, g.n))
    o = reverse_cuthill_mckee(A, symmetric_mode=True)
    ref = np.empty(g.n, dtype=np.int64)
    ref[o] = np.arange(g.n)
    theirs = _bandwidth(g, ref)
    print(f"bandwidth: points {_bandwidth(g, np.arange(g.n))}, ours {ours}, scipy {theirs}")
    assert ours <= 1.25 * theirs
    assert ours < 0.05 * g.n


def test_rcm_components_and_isolated_nodes():
    """Two shuffled paths and three isolated nodes: every component occupies a contiguous id range
    (a breadth-first sweep finishes one component before it starts the next)."""
    i = np.concatenate([np.arange(0, 99), np.arange(100, 179)])
    j = i + 1
    g = _shuffled(gen.csr_from_edges(183, i, j, lambda lo, hi: np.ones(len(lo), dtype=np.float32)), 3)
    perm = pspec.rcm_order(g.rowptr, g.col)
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components

    _, comp = connected_components(csr_matrix((g.w, g.col, g.rowptr), shape=(g.n, g.n)), directed=False)
    for c in np.unique(comp):
        ids = np.sort(perm[comp == c])
        assert ids[-1] - ids[0] == len(ids) - 1
    assert _bandwidth(g, perm) == 1


def test_rcm_rejects_bad_csr():
    with pytest.raises(pspec.PSpecError):
        pspec.rcm_order(np.array([0, 2, 1]), np.array([1, 0], dtype=np.int32))
    with pytest.raises(pspec.PSpecError):
        pspec.rcm_order(np.array([0, 1, 2]), np.array([1, 5], dtype=np.int32))
    assert len(pspec.rcm_order(np.array([0]), np.array([], dtype=np.int32))) == 0


def test_relabel_moves_edges_and_points():
    g = gen.delaunay(500, seed=1)
    perm = np.random.default_rng(5).permutation(g.n)
    h = gen.relabel(g, perm)
    assert np.array_equal(h.to_dense()[np.ix_(perm, perm)], g.to_dense())
    assert np.array_equal(h.meta["points"][perm], g.meta["points"])
