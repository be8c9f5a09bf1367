"""Seeded synthetic inputs: graphs in symmetric CSR form and dense n x k blocks.

This module only draws inputs.  It holds none of the method's arithmetic (no objective, no
p-Laplacian, no projection), so the FP64 oracle and the HIP path can both be fed from it
without sharing any computation.

The paper evaluates on SuiteSparse Delaunay triangulations (Section 3), which are not
available here; the generators below are synthetic stand-ins with the shapes of the stated
workloads:

* ``sbm_bernoulli``  stochastic block model, Bernoulli trial on every node pair (small n);
* ``knn_mixture``    symmetrised k-nearest-neighbour graph of a 2-D Gaussian mixture;
* ``grid3d``         3-D 6-neighbour grid, lexicographic node order;
* ``sbm_edges``      stochastic block model drawn edge by edge, block-contiguous node ids;
* ``rmat``           R-MAT recursive-matrix graph, unpermuted ids.

Every graph is returned as symmetric CSR: both directions of each undirected edge stored,
no self-loops, no duplicate entries, columns ascending within a row, int64 row pointers,
int32 column indices and float32 weights.  A weight is drawn once per undirected edge, so
w_ij == w_ji bit for bit.  Where a weight is random it comes from a counter-based hash of
the (seed, min(i,j), max(i,j)) triple, which makes duplicate draws of the same edge carry the
same value and keeps the generator independent of the order of the edge list.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_GRAPH = 2605
SEED_U = 1
SEED_V = 2


@dataclass
class Graph:
    """Symmetric CSR graph: row i's neighbours are col[rowptr[i]:rowptr[i+1]]."""

    n: int
    rowptr: np.ndarray  # int64, n + 1
    col: np.ndarray  # int32, nnz
    w: np.ndarray  # float32, nnz
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.rowptr)

    def to_dense(self) -> np.ndarray:
        """Dense float64 weight matrix (small graphs only)."""
        W = np.zeros((self.n, self.n), dtype=np.float64)
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        W[rows, self.col] = self.w
        return W


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser on uint64 arrays (Steele, Lea, Flood 2014)."""
    x = x.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        x += np.uint64(0x9E3779B97F4A7C15)
        x ^= x >> np.uint64(30)
        x *= np.uint64(0xBF58476D1CE4E5B9)
        x ^= x >> np.uint64(27)
        x *= np.uint64(0x94D049BB133111EB)
        x ^= x >> np.uint64(31)
    return x


def edge_uniform(seed: int, lo_id: np.ndarray, hi_id: np.ndarray, lo: float, hi: float) -> np.ndarray:
    """Per-undirected-edge uniform weights in [lo, hi), from a hash of (seed, min id, max id).

    The uniform variate has 24 random bits, so lo + (hi - lo) * u is formed in float64 and
    rounded to float32 once.
    """
    key = (lo_id.astype(np.uint64) << np.uint64(32)) | hi_id.astype(np.uint64)
    with np.errstate(over="ignore"):
        key ^= np.uint64((seed * 0xD1B54A32D192ED03) & 0xFFFFFFFFFFFFFFFF)
    u = (_splitmix64(key) >> np.uint64(40)).astype(np.float64) * (1.0 / (1 << 24))
    return (lo + (hi - lo) * u).astype(np.float32)


def delaunay(n: int, seed: int = SEED_GRAPH) -> Graph:
    """Delaunay triangulation of n uniform random points in the unit square, unit weights (a
    stand-in for triangulation graphs: planar, connected, mean degree just under 6)."""
    from scipy.spatial import Delaunay

    pts = np.random.default_rng(seed).random((n, 2))
    tri = Delaunay(pts).simplices.astype(np.int64)
    i = np.concatenate([tri[:, 0], tri[:, 1], tri[:, 2]])
    j = np.concatenate([tri[:, 1], tri[:, 2], tri[:, 0]])
    g = csr_from_edges(n, i, j, lambda lo, hi: np.ones(len(lo), dtype=np.float32), name=f"delaunay{n}")
    g.meta["points"] = pts
    return g


def relabel(g: Graph, perm: np.ndarray, name: str = "relabelled") -> Graph:
    """The same graph with node ids relabelled (new id = perm[old]), weights carried with their
    edges; columns ascend within each row of the result."""
    perm = np.asarray(perm, dtype=np.int64)
    deg = np.diff(g.rowptr)
    rows = np.repeat(perm, deg)
    cols = perm[g.col.astype(np.int64)]
    key = rows * g.n + cols
    order = np.argsort(key, kind="stable")
    new_rows = rows[order]
    rowptr = np.zeros(g.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(new_rows, minlength=g.n), out=rowptr[1:])
    meta = dict(g.meta)
    if "points" in meta:
        pts = np.empty_like(meta["points"])
        pts[perm] = meta["points"]
        meta["points"] = pts
    return Graph(g.n, rowptr, cols[order].astype(np.int32), g.w[order], name=f"{g.name}-{name}", meta=meta)


def induced(g: Graph, keep: np.ndarray, name: str = "induced") -> tuple[Graph, np.ndarray]:
    """The subgraph on the nodes with keep[i] true, renumbered in node order; returns it and the
    original ids of its nodes.  Edges to dropped nodes are removed."""
    keep = np.asarray(keep, dtype=bool)
    ids = np.flatnonzero(keep).astype(np.int64)
    new_id = np.full(g.n, -1, dtype=np.int64)
    new_id[ids] = np.arange(len(ids))
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    e = keep[rows] & keep[g.col]
    r, c = new_id[rows[e]], new_id[g.col[e].astype(np.int64)]
    rowptr = np.zeros(len(ids) + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=len(ids)), out=rowptr[1:])
    meta = {k: v for k, v in g.meta.items() if k != "points"}
    if "points" in g.meta:
        meta["points"] = g.meta["points"][ids]
    return Graph(len(ids), rowptr, c.astype(np.int32), g.w[e], name=f"{g.name}-{name}", meta=meta), ids


def permute(g: Graph, seed: int) -> Graph:
    """The same graph with node ids relabelled by a seeded random permutation (new id = perm[old])."""
    perm = np.random.default_rng(seed).permutation(g.n).astype(np.int64)
    h = relabel(g, perm, "permuted")
    h.meta["permutation_seed"] = seed
    return h


def csr_from_edges(n: int, i: np.ndarray, j: np.ndarray, weight_fn, name: str = "", meta=None) -> Graph:
    """Build symmetric CSR from an undirected edge list (any order, duplicates and loops allowed).

    Self-loops are dropped; duplicates are merged (all copies of one undirected edge carry the
    same weight, see ``weight_fn``); both directions are stored; columns ascend within a row.
    ``weight_fn(lo, hi)`` returns float32 weights for canonical pairs lo < hi.
    """
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    keep = i != j
    i, j = i[keep], j[keep]
    lo = np.minimum(i, j)
    hi = np.maximum(i, j)
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key - lo * n
    w_und = weight_fn(lo, hi).astype(np.float32)
    # mirror: directed key row * n + col; sort gives CSR order (rows ascending, cols ascending)
    dkey = np.concatenate([lo * n + hi, hi * n + lo])
    order = np.argsort(dkey, kind="stable") if len(dkey) < (1 << 22) else None
    if order is not None:
        dkey = dkey[order]
        w = np.concatenate([w_und, w_und])[order]
    else:
        dkey.sort()
        rows = dkey // n
        cols = dkey - rows * n
        w = weight_fn(np.minimum(rows, cols), np.maximum(rows, cols)).astype(np.float32)
    rows = dkey // n
    cols = (dkey - rows * n).astype(np.int32)
    counts = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return Graph(n=n, rowptr=rowptr, col=cols, w=np.ascontiguousarray(w, dtype=np.float32), name=name,
                 meta=dict(meta or {}))


def sbm_bernoulli(n: int = 1000, blocks: int = 4, p_in: float = 0.05, p_out: float = 0.002,
                  seed: int = SEED_GRAPH, weight: float = 1.0) -> Graph:
    """SBM with equal contiguous blocks; every pair i < j is an edge with prob p_in / p_out."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, k=1)
    bs = n // blocks
    same = (np.minimum(iu // bs, blocks - 1)) == (np.minimum(ju // bs, blocks - 1))
    prob = np.where(same, p_in, p_out)
    hit = rng.random(len(iu)) < prob
    return csr_from_edges(n, iu[hit], ju[hit], lambda lo, hi: np.full(len(lo), weight, np.float32),
                          name=f"sbm{n}", meta=dict(blocks=blocks, p_in=p_in, p_out=p_out))


def knn_mixture(n: int = 100_000, comps: int = 8, knn: int = 10, sigma: float = 1.0, box: float = 20.0,
                seed: int = SEED_GRAPH) -> Graph:
    """kNN graph of a 2-D Gaussian mixture, symmetrised by union, w = exp(-d^2 / s^2).

    Points are ordered by component; s is the median over points of the distance to the
    knn-th neighbour.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    centres = rng.uniform(-box, box, size=(comps, 2))
    per = n // comps
    counts = np.full(comps, per)
    counts[: n - per * comps] += 1
    pts = np.concatenate([centres[c] + sigma * rng.standard_normal((counts[c], 2)) for c in range(comps)])
    tree = cKDTree(pts)
    d, idx = tree.query(pts, k=knn + 1)
    s = float(np.median(d[:, knn]))
    i = np.repeat(np.arange(n), knn)
    j = idx[:, 1:].reshape(-1)

    def wfn(lo, hi):
        dd = np.sum((pts[lo] - pts[hi]) ** 2, axis=1)
        return np.exp(-dd / (s * s)).astype(np.float32)

    labels = np.repeat(np.arange(comps), counts)
    return csr_from_edges(n, i, j, wfn, name=f"knn{n}", meta=dict(s=s, labels=labels))


def grid3d(side: int = 128) -> Graph:
    """Non-periodic 3-D 6-neighbour grid, node id x + side*y + side^2*z, unit weights."""
    n = side ** 3
    ids = np.arange(n, dtype=np.int64).reshape(side, side, side)  # [z, y, x]
    pairs = []
    pairs.append((ids[:, :, :-1].ravel(), ids[:, :, 1:].ravel()))
    pairs.append((ids[:, :-1, :].ravel(), ids[:, 1:, :].ravel()))
    pairs.append((ids[:-1, :, :].ravel(), ids[1:, :, :].ravel()))
    i = np.concatenate([p[0] for p in pairs])
    j = np.concatenate([p[1] for p in pairs])
    return csr_from_edges(n, i, j, lambda lo, hi: np.ones(len(lo), np.float32), name=f"grid{side}^3")


def sbm_edges(n: int = 8_000_000, blocks: int = 16, m_intra: int = 43_200_000, m_inter: int = 4_800_000,
              wlo: float = 0.5, whi: float = 1.5, seed: int = SEED_GRAPH) -> Graph:
    """SBM drawn edge by edge with block-contiguous node ids.

    m_intra draws with both endpoints uniform in one block (m_intra / blocks per block) and
    m_inter draws whose endpoints are uniform in two different blocks; loops and duplicate
    draws are removed; weights uniform in [wlo, whi).
    """
    rng = np.random.default_rng(seed)
    bs = n // blocks
    per = m_intra // blocks
    b = np.repeat(np.arange(blocks, dtype=np.int64), per)
    i1 = b * bs + rng.integers(0, bs, size=len(b))
    j1 = b * bs + rng.integers(0, bs, size=len(b))
    bi = rng.integers(0, blocks, size=m_inter)
    bj = (bi + rng.integers(1, blocks, size=m_inter)) % blocks
    i2 = bi * bs + rng.integers(0, bs, size=m_inter)
    j2 = bj * bs + rng.integers(0, bs, size=m_inter)
    i = np.concatenate([i1, i2])
    j = np.concatenate([j1, j2])
    del i1, j1, i2, j2, b, bi, bj
    return csr_from_edges(n, i, j, lambda lo, hi: edge_uniform(seed, lo, hi, wlo, whi),
                          name=f"sbm{n}", meta=dict(blocks=blocks, labels_block=bs))


def rmat(scale: int = 22, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         wlo: float = 0.1, whi: float = 1.0, seed: int = SEED_GRAPH) -> Graph:
    """R-MAT graph (Chakrabarti, Zhan, Faloutsos 2004), no noise, unpermuted ids.

    edge_factor * 2^scale draws; at each of the scale levels a quadrant is chosen with
    probabilities (a, b, c, d = 1 - a - b - c); loops removed, symmetrised, deduplicated.
    """
    rng = np.random.default_rng(seed)
    n = 1 << scale
    m = edge_factor * n
    i = np.zeros(m, dtype=np.int64)
    j = np.zeros(m, dtype=np.int64)
    t_ab, t_abc = a + b, a + b + c
    for level in range(scale):
        r = rng.random(m, dtype=np.float32)
        bit = np.int64(1 << (scale - 1 - level))
        row_hi = r >= t_ab  # quadrants c, d
        col_hi = ((r >= a) & (r < t_ab)) | (r >= t_abc)  # quadrants b, d
        i += row_hi * bit
        j += col_hi * bit
    del r, row_hi, col_hi
    return csr_from_edges(n, i, j, lambda lo, hi: edge_uniform(seed, lo, hi, wlo, whi),
                          name=f"rmat{scale}", meta=dict(a=a, b=b, c=c))


def block(n: int, k: int, seed: int) -> np.ndarray:
    """n x k float32 block with N(0, 1) entries, rows drawn in row-major order."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, k), dtype=np.float64).astype(np.float32)


# The five workloads with their stated recipes.  Values: graph builder, k, p levels, eps.
CONFIGS = {
    "sbm1000": dict(graph=lambda: sbm_bernoulli(1000, 4, 0.05, 0.002), k=4, p=(2.0, 1.6, 1.3, 1.1), eps=1e-8),
    "knn100k": dict(graph=lambda: knn_mixture(100_000, 8, 10, 1.0, 20.0), k=8, p=(1.3,), eps=1e-8),
    "grid128": dict(graph=lambda: grid3d(128), k=8, p=(1.2,), eps=1e-8),
    "sbm8m": dict(graph=lambda: sbm_edges(8_000_000, 16, 43_200_000, 4_800_000, 0.5, 1.5), k=16, p=(1.1,),
                  eps=1e-8),
    "rmat22": dict(graph=lambda: rmat(22, 16, 0.57, 0.19, 0.19, 0.1, 1.0), k=32, p=(1.05,), eps=1e-8),
}
