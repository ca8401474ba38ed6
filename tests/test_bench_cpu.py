"""Host-side pieces of bench.py: the per-iteration algorithmic byte count and
the trajectory-error comparison used for the precision forms (CPU only)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_iteration_bytes_10000():
    m = n = 10000
    k, q = 2_000_000, 2
    # bf16 iteration: 8 panel passes of 200 MB, the 400 MB residual read,
    # 8 x 16 MB of S corrections, 40 MB of S write and candidates
    assert bench.iteration_bytes(m, n, k, q, 2) == 8 * 200e6 + 400e6 + 128e6 + 40e6
    # FP32 plain: 9 reads of 400 MB plus the same S traffic
    assert bench.iteration_bytes(m, n, k, q, 4) == 9 * 400e6 + 128e6 + 40e6
    # refinement: 4 bf16 subspace passes, the last subspace pass and the
    # 3-pass B chain in FP32
    assert bench.iteration_bytes(m, n, k, q, 2, refine=True) == \
        4 * 200e6 + 4 * 400e6 + 400e6 + 168e6


def test_roofline_fraction_formula():
    stats = [{"name": "k", "launches": 10, "total_ms": 1.0, "bytes_per_launch": 2e8}]
    r = bench.roofline_of(stats, 10000, 10000, 2_000_000, 2, 20, 20 * 1.357, True)
    b = (19 * 2.168e9 + 2.968e9) / 20
    assert abs(r["algorithmic_bytes_per_iteration"] - b) < 1
    assert abs(r["frac"] - b / 1.357e-3 / 8e12) < 1e-4


def test_trajectory_errors_identity_and_swap():
    rng = np.random.default_rng(3)
    m, n, r, k = 60, 40, 3, 50
    U, V = rng.standard_normal((m, r)), rng.standard_normal((n, r))
    X = U @ V.T + rng.standard_normal((m, n)) * 0.01
    L = U @ V.T
    R = X - L
    order = np.argsort(-np.abs(R).ravel(), kind="stable")
    idx = np.sort(order[:k])
    S = np.zeros(m * n)
    S[idx] = R.ravel()[idx]
    S = S.reshape(m, n)
    thr = float(np.abs(R.ravel()[order[k - 1]]))
    e = bench.trajectory_errors(X, U, V, idx, R.ravel()[idx], thr, L, S, thr)
    assert e["rel_L"] == 0 and e["rel_S"] == 0 and e["swaps"] == 0 and e["rel_obj"] == 0
    # swap the k-th entry for the (k+1)-th: two swaps at the threshold
    idx2 = np.sort(np.concatenate([order[:k - 1], order[k:k + 1]]))
    e = bench.trajectory_errors(X, U, V, idx2, R.ravel()[idx2],
                                float(np.abs(R.ravel()[order[k]])), L, S, thr)
    assert e["swaps"] == 2 and e["swaps_gpu_only"] == 1 and e["swaps_oracle_only"] == 1
    assert e["common"] == k - 1 and e["rel_S_common"] == 0 and e["swaps_within_band"]
