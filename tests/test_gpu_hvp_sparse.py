"""GPU: pspec_hvp_sparse (Algorithm 1 read with sparse D[l], H[l]: the Hessian without its rank-2
part) against the oracle's sparse operator, element by element, on an SBM graph and an R-MAT graph
with heavy and split rows; its G and F are pspec_hvp's, bit for bit."""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_2605_26975_amd import gen, pspec
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

GRAPHS = {
    "sbm1000": lambda: gen.sbm_bernoulli(1000, 4, 0.05, 0.002),
    "rmat13": lambda: gen.rmat(13, 16, 0.57, 0.19, 0.19, 0.1, 1.0, seed=2),
}


@pytest.mark.parametrize("gname", sorted(GRAPHS))
@pytest.mark.parametrize("k", [4, 16, 33])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_hvp_sparse_matches_oracle(gname, k, dtype):
    p, eps = 1.3, 1e-8
    print(f"[case] hvp_sparse {gname} k={k} {dtype}", flush=True)
    g = GRAPHS[gname]()
    U, V = gu.inputs(g.n, k)
    dg = gu.device_graph(g, k)
    Ud = torch.as_tensor(U).to(dtype).cuda()
    Vd = torch.as_tensor(V).to(dtype).cuda()
    HVs, Gs, Fs = pspec.hvp(dg, Ud, Vd, p, eps, sparse_only=True)
    HV, G, F = pspec.hvp(dg, Ud, Vd, p, eps)
    assert torch.equal(Gs, G) and torch.equal(Fs, F)
    ref = orc.default().hvp_sparse(g.rowptr, g.col, g.w.astype(np.float64), U.astype(np.float64),
                                   V.astype(np.float64), p, eps)
    _, _, SHs = gu.oracle_scales(g, U, V, p, eps, sparse=True)
    HVh = HVs.double().cpu().numpy()
    t = gu.TOLS[dtype]
    err, cmax, ewr = gu.rel(HVh, ref), gu.colmax(HVh, ref), gu.ew(HVh, ref, SHs)
    print(f"rel err {err:.2e}, column max {cmax:.2e}, element-wise {ewr:.2e}")
    assert err <= t["norm"] and cmax <= t["norm"] and ewr <= t["tau"]
    # the two operators differ exactly by the rank-2 term: never equal unless it vanishes
    assert not torch.equal(HVs, HV)
