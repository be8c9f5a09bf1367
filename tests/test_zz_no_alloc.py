"""GPU: pspec_rhvp_static, the allocation-free variant of pspec_rhvp (its dense workspace is the
library's per-GPU static scratch), called through the C ABI and compared with pspec_rhvp bit for
bit on two calls in a row, the second with a smaller graph and block."""
import numpy as np
import pytest
import torch

from paper_2605_26975_amd import gen, pspec
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _tangent(n, k, seed, dtype):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, k)))
    V0 = rng.standard_normal((n, k))
    V = V0 - U @ (U.T @ V0)
    P = torch.empty((n, 2 * k), dtype=dtype, device="cuda")
    P[:, :k] = torch.as_tensor(U).to(dtype)
    P[:, k:] = torch.as_tensor(V).to(dtype)
    return P[:, :k], P[:, k:]


def _outputs(U):
    n, k = U.shape
    return (torch.empty_like(U), torch.empty_like(U), torch.empty((k, k), dtype=torch.float64, device=U.device),
            torch.empty(k, dtype=torch.float64, device=U.device))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_rhvp_static_matches_rhvp_on_two_calls(dtype):
    cases = [("sbm30k k=32", gen.sbm_edges(30_000, 8, 150_000, 20_000, 0.5, 1.5, seed=12), 32),
             ("sbm1000 k=5", gen.sbm_bernoulli(1000, 4, 0.05, 0.002), 5)]
    p, eps = 1.3, 1e-8
    for name, g, k in cases:
        print(f"[case] rhvp_static {name} {dtype}", flush=True)
        dg = gu.device_graph(g, k)
        U, V = _tangent(g.n, k, seed=k, dtype=dtype)
        ref = pspec.rhvp(dg, U, V, p, eps)
        out = _outputs(U)
        for t in out:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        allocs = torch.cuda.memory_stats()["allocation.all.allocated"]
        got = pspec.rhvp_static(dg, U, V, p, eps, *out)
        torch.cuda.synchronize()
        # no device allocation through torch on the call's path (the count of allocations ever made)
        assert torch.cuda.memory_stats()["allocation.all.allocated"] == allocs
        for nm, a, b in zip(("RH", "RG", "MG", "F_col"), got, ref):
            assert torch.equal(a, b), (name, nm)
        del got, ref, out


def test_rhvp_static_rejects_wide_blocks():
    g = gen.sbm_bernoulli(1000, 4, 0.05, 0.002)
    k = pspec.STATIC_K_MAX + 1
    dg = gu.device_graph(g, k)
    U, V = _tangent(g.n, k, seed=1, dtype=torch.float32)
    with pytest.raises(pspec.PSpecError) as ei:
        pspec.rhvp_static(dg, U, V, 1.3, 1e-8, *_outputs(U))
    assert ei.value.status == 2 and "static" in str(ei.value)
