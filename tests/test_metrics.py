"""Clustering diagnostics against hand-counted examples and their defining properties."""
import numpy as np
import pytest

from paper_1403_7394_amd import metrics


def test_purity_hand_example():
    # clusters {0,1,2}: classes a,a,b -> 2; {3,4}: b,b -> 2; {5}: c -> 1; purity 5/6
    labels = [7, 7, 7, 3, 3, 9]
    truth = ["a", "a", "b", "b", "b", "c"]
    assert metrics.purity(labels, truth) == pytest.approx(5 / 6, abs=0)


def test_purity_extremes():
    truth = np.repeat(np.arange(4), 5)
    assert metrics.purity(truth * 10, truth) == 1.0                       # same partition
    assert metrics.purity(np.arange(20), truth) == 1.0                    # singletons are pure
    assert metrics.purity(np.zeros(20, int), truth) == pytest.approx(0.25)  # one cluster: largest class share
    with pytest.raises(ValueError):
        metrics.purity([], [])


def test_adjusted_rand_index_hand_example_and_properties():
    # a = {0,1},{2,3}; b = {0,1,2},{3}: pairs agreeing in both: (0,1) only.
    # sum_ij C(n_ij,2) = 1; sum_a = 1 + 1 = 2; sum_b = 3 + 0 = 3; total C(4,2) = 6
    # expected = 2*3/6 = 1; max = 2.5 -> ARI = (1 - 1) / (2.5 - 1) = 0
    assert metrics.adjusted_rand_index([0, 0, 1, 1], [0, 0, 0, 1]) == pytest.approx(0.0, abs=1e-15)
    x = np.random.default_rng(1).integers(0, 5, 200)
    assert metrics.adjusted_rand_index(x, x) == 1.0
    assert metrics.adjusted_rand_index(x, (x + 3) % 5) == 1.0            # relabelling
    y = np.random.default_rng(2).integers(0, 5, 200)
    assert metrics.adjusted_rand_index(x, y) == pytest.approx(metrics.adjusted_rand_index(y, x))
