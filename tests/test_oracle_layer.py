"""Pins of the layer oracle: its autograd gradient against central finite
differences of the same frozen-mask forward (FP64), on the small layer
configuration (64 x 48, r = 2, k = 150, q = 1, T = 10)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import godec_layer_ref as lr
from oracle import godec_ref as g
from paper_1309_0302_amd import workloads as wl


def small_case(seed=1006, q=1, T=10):
    w = wl.tiny(64, 48, 2, rho=150 / (64 * 48), seed=seed, dtype=np.float64, noise_std=1e-3)
    A1 = np.random.default_rng(seed).standard_normal((48, 2))
    tr = g.godec_brp(w.X, 2, 150, q, A1, T, keep_supports=True)
    rng = np.random.default_rng(seed + 1)
    dL = rng.standard_normal(w.X.shape)
    dS = rng.standard_normal(w.X.shape)
    return w.X, A1, tr.supports, dL, dS


def test_frozen_forward_matches_the_oracle_loop():
    X, A1, masks, _, _ = small_case()
    tr = g.godec_brp(X, 2, 150, 1, A1, len(masks))
    L, S = lr.layer_forward(torch.tensor(X), torch.tensor(A1), 1, masks)
    assert g.rel_fro(L.numpy(), tr.L) < 1e-12
    assert g.rel_fro(S.numpy(), tr.S) < 1e-12


@pytest.mark.parametrize("q", [0, 1, 2])
def test_autograd_gradient_matches_finite_differences(q):
    X, A1, masks, dL, dS = small_case(q=q, T=10 if q == 1 else 4)
    grad = lr.layer_grad(X, A1, q, masks, dL, dS)
    rng = np.random.default_rng(7)
    h = 1e-6 * np.abs(X).max()
    worst = 0.0
    for _ in range(12):
        V = rng.standard_normal(X.shape)
        fd = (lr.layer_value(X + h * V, A1, q, masks, dL, dS)
              - lr.layer_value(X - h * V, A1, q, masks, dL, dS)) / (2 * h)
        ad = float(np.sum(grad * V))
        worst = max(worst, abs(fd - ad) / max(abs(ad), 1e-300))
    assert worst < 1e-6, worst


def test_finite_differences_catch_a_wrong_gradient():
    """A gradient that ignores the mask term of S_T is rejected by the pin."""
    X, A1, masks, dL, dS = small_case(T=3)
    good = lr.layer_grad(X, A1, 1, masks, dL, dS)
    bad = lr.layer_grad(X, A1, 1, masks, dL, np.zeros_like(dS))
    rng = np.random.default_rng(8)
    V = rng.standard_normal(X.shape)
    h = 1e-6 * np.abs(X).max()
    fd = (lr.layer_value(X + h * V, A1, 1, masks, dL, dS)
          - lr.layer_value(X - h * V, A1, 1, masks, dL, dS)) / (2 * h)
    assert abs(fd - np.sum(good * V)) < 1e-6 * abs(fd)
    assert abs(fd - np.sum(bad * V)) > 1e-3 * abs(fd)
