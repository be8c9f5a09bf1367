"""GPU: the k-means step (pspec_kmeans_step) against the oracle's step, and the Lloyd driver against
the oracle's Lloyd iterations.  Labels and distances are compared bit for bit (both sides sum the
squared coordinate differences in order, in FP64, without fused multiply-adds); the cluster sums are
FP64 sums of the same terms in different orders, compared within the bound 2 (m - 1) u sum |x| that
any two summation orders of m terms satisfy (u = 2^-53)."""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_2605_26975_amd import driver, gen, pspec

pytestmark = pytest.mark.gpu

U53 = 2.0 ** -53


def _centroids(X, c, seed):
    rng = np.random.default_rng(seed)
    idx = rng.choice(X.shape[0], size=c, replace=X.shape[0] < c)
    return X[idx].astype(np.float64) + 0.1 * rng.standard_normal((c, X.shape[1]))


def _device_block(X, dtype, pad):
    """X as a device block of the given dtype, with `pad` extra columns in its rows (ldx = d + pad)."""
    n, d = X.shape
    buf = torch.zeros((n, d + pad), dtype=dtype, device="cuda")
    buf[:, :d] = torch.as_tensor(X, dtype=dtype)
    return buf[:, :d]


def _check_step(X, C, dtype, pad=0):
    n, d = X.shape
    c = C.shape[0]
    Xd = _device_block(X, dtype, pad)
    Xh = Xd.double().cpu().numpy()  # the values the kernel sees
    dist = torch.empty(n, dtype=torch.float64, device="cuda")
    labels, _, stats = pspec.kmeans_step(Xd, torch.as_tensor(C).cuda(), dist=dist)
    lo, do, so = orc.kmeans_step(Xh, C)
    assert np.array_equal(labels.cpu().numpy(), lo)
    assert np.array_equal(dist.cpu().numpy(), do)
    s = stats.cpu().numpy()
    assert np.array_equal(s[:, d], so[:, d])
    cnt = so[:, d]
    absx = np.zeros((c, d))
    np.add.at(absx, lo, np.abs(Xh))
    bound = 2.0 * np.maximum(cnt - 1, 0)[:, None] * U53 * absx * (1 + 1e-6)
    assert np.all(np.abs(s[:, :d] - so[:, :d]) <= bound)
    dsum = np.zeros(c)
    np.add.at(dsum, lo, do)
    assert np.all(np.abs(s[:, d + 1] - so[:, d + 1]) <= 2.0 * np.maximum(cnt - 1, 0) * U53 * dsum * (1 + 1e-6))
    return s


CASES = [(1, 1, 1), (63, 3, 2), (1000, 4, 4), (5000, 5, 7), (20000, 8, 3), (4099, 13, 32), (3000, 16, 16),
         (2000, 32, 32), (300001, 4, 4)]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("n,d,c", CASES)
def test_kmeans_step_matches_oracle(dtype, n, d, c):
    print(f"[case] kmeans_step n={n} d={d} c={c} {dtype}", flush=True)
    X = gen.block(n, d, gen.SEED_U)
    _check_step(X, _centroids(X, c, 5), dtype)


@pytest.mark.parametrize("d,pad", [(4, 1), (5, 3), (16, 2)])
def test_kmeans_step_strided_rows(d, pad):
    print(f"[case] kmeans_step strided d={d} ldx={d + pad}", flush=True)
    X = gen.block(7000, d, gen.SEED_V)
    _check_step(X, _centroids(X, 6, 9), torch.float32, pad)


def test_kmeans_step_exact_ties_go_to_the_lower_index():
    """Integer coordinates make every distance exact, so rows halfway between centroids tie exactly;
    both sides must pick the lower centroid index."""
    rng = np.random.default_rng(2)
    X = rng.integers(-3, 4, size=(5000, 2)).astype(np.float64)
    C = np.array([[0.0, 0.0], [2.0, 0.0], [0.0, 2.0], [-2.0, 0.0], [0.0, 0.0]])  # centroid 4 repeats 0
    s = _check_step(X, C, torch.float64)
    assert s[4, 2] == 0.0  # the duplicate centroid never wins a tie


def test_kmeans_step_full_size_block():
    """U of the 2^21-node Delaunay graph, k = 4: the clustering the pipeline runs."""
    print("[case] kmeans_step n=2^21+5 d=4 c=4", flush=True)
    X = gen.block((1 << 21) + 5, 4, gen.SEED_U)
    _check_step(X, _centroids(X, 4, 1), torch.float32)


def test_kmeans_step_empty_and_reproducible():
    C = torch.as_tensor(np.eye(3)).cuda()
    X0 = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    stats = torch.full((3, 5), 7.0, dtype=torch.float64, device="cuda")
    pspec.kmeans_step(X0, C, stats=stats)
    assert torch.all(stats == 0.0)
    X = torch.as_tensor(gen.block(100000, 3, gen.SEED_U)).cuda()
    a = pspec.kmeans_step(X, C)[2].clone()
    b = pspec.kmeans_step(X, C)[2]
    assert torch.equal(a, b)


def test_lloyd_matches_the_oracle():
    rng = np.random.default_rng(4)
    centres = rng.normal(scale=4.0, size=(6, 5))
    truth = rng.integers(0, 6, 30000)
    X = (centres[truth] + rng.standard_normal((30000, 5))).astype(np.float64)
    C0 = X[rng.choice(30000, 6, replace=False)]
    Xd = torch.as_tensor(X).cuda()
    lab, C, inertia, steps = driver.lloyd_gpu(Xd, C0)
    lo, Co, io, so = orc.lloyd(X, C0)
    print(f"steps gpu {steps} oracle {so}")
    assert np.array_equal(lab.cpu().numpy(), lo)
    assert steps == so
    assert np.allclose(C, Co, rtol=1e-12, atol=1e-13)
    assert abs(inertia - io) <= 1e-10 * io


def test_kmeans_separated_blobs():
    rng = np.random.default_rng(0)
    centres = np.array([[0, 0], [10, 0], [0, 10], [10, 10]], dtype=float)
    truth = np.repeat(np.arange(4), 200)
    X = centres[truth] + rng.standard_normal((800, 2))
    labels, C, inertia = driver.kmeans_gpu(torch.as_tensor(X, dtype=torch.float32).cuda(), 4, seed=3)
    assert driver.matched_accuracy(labels, truth) == 1.0
    # every point is closer to its own centre than to any other: inertia near 2 per point
    assert 1.5 * 800 < inertia < 2.5 * 800
