"""Host-side pieces of the driver (CPU only): RCut, label matching, p schedule."""
import numpy as np
import pytest

from paper_2605_26975_amd import driver
from tests import pins


def test_rcut_hand_example():
    """Two triangles joined by one edge of weight 0.5, split into the two triangles:
    cut(C1) = cut(C2) = 0.5, |C1| = |C2| = 3, RCut = 0.5/3 + 0.5/3 (Section 3.1 definition)."""
    W = np.zeros((6, 6))
    for a, b in ((0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)):
        W[a, b] = W[b, a] = 1.0
    W[2, 3] = W[3, 2] = 0.5
    rp, c, w = pins.csr_from_dense(W)
    assert abs(driver.rcut(rp, c, w, np.array([0, 0, 0, 1, 1, 1])) - 1.0 / 3.0) < 1e-15
    # a worse split: {0,1} vs the rest -> cut = w02 + w12 = 2, RCut = 2/2 + 2/4
    assert abs(driver.rcut(rp, c, w, np.array([0, 0, 1, 1, 1, 1])) - 1.5) < 1e-15


def test_matched_accuracy_is_permutation_invariant():
    a = np.array([0, 0, 1, 1, 2, 2])
    b = np.array([2, 2, 0, 0, 1, 1])
    assert driver.matched_accuracy(a, b) == 1.0
    c = np.array([2, 2, 0, 1, 1, 1])
    assert abs(driver.matched_accuracy(a, c) - 5 / 6) < 1e-15


def test_p_levels():
    assert driver.p_levels(2.0) == [2.0]
    assert driver.p_levels(1.1) == [2.0, 1.8, 1.6, 1.4, 1.2, 1.1]
    assert driver.p_levels(1.2) == [2.0, 1.8, 1.6, 1.4, 1.2]


def test_cluster_rejects_unknown_method():
    with pytest.raises(ValueError):
        driver.cluster(None, None, 2, 1.5, method="bfgs")
