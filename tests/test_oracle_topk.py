"""Pins for the oracle's hard threshold (Eq. 4, Algorithm 1 S-update)."""
import numpy as np
import pytest

from oracle import godec_ref as g


def brute(R, k):
    """Full stable sort by (|value| desc, linear index asc), first k, nonzero."""
    a = np.abs(R).ravel()
    order = sorted(range(a.size), key=lambda i: (-a[i], i))
    sel = [i for i in order[:k] if a[i] != 0]
    return np.array(sorted(sel), dtype=np.int64)


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_tie_heavy(seed):
    rng = np.random.default_rng(seed)
    m, n = rng.integers(1, 9), rng.integers(1, 9)
    R = rng.integers(-3, 4, size=(m, n)).astype(np.float64)   # many ties, zeros
    for k in range(0, m * n + 3):
        idx, val = g.hard_threshold(R, k)
        assert np.array_equal(idx, brute(R, k))
        assert np.array_equal(val, R.ravel()[idx])


def test_eq4_optimality_condition():
    rng = np.random.default_rng(1)
    R = rng.standard_normal((40, 30))
    for k in (1, 17, 300, 1199):
        idx, val = g.hard_threshold(R, k)
        mask = np.zeros(R.size, bool)
        mask[idx] = True
        a = np.abs(R).ravel()
        assert idx.size == k
        assert a[mask].min() >= a[~mask].max()
        # S minimises ||R - S|| over card(S) <= k: the residual is the rest
        S = g.dense_from_support(R.shape, idx, val)
        assert np.isclose(np.sum((R - S) ** 2), np.sum(a[~mask] ** 2))


def test_zeros_excluded_and_signs_kept():
    R = np.array([[0.0, -2.0], [0.0, 1.0]])
    idx, val = g.hard_threshold(R, 4)
    assert idx.tolist() == [1, 3] and val.tolist() == [-2.0, 1.0]
    idx, val = g.hard_threshold(np.zeros((3, 3)), 2)
    assert idx.size == 0


def test_negative_zero_counts_as_zero():
    R = np.array([[-0.0, 0.0, 3.0]])
    idx, _ = g.hard_threshold(R, 3)
    assert idx.tolist() == [2]
