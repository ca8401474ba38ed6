"""Pins of the GoDec matrix-completion oracle (Sec. 2: the cardinality
constraint replaced by a fixed support set).  CPU only.

- A rank-r matrix is recovered from 70 % of its entries to 1e-12 (the
  definition of completion: the only rank-r matrix agreeing with the
  observed entries, for random supports at this sampling rate).
- The imputation invariant: D = X - S_t equals X on the observed entries
  and L_t on the unobserved ones.
- The S step zeroes the residual on the support (its exact minimiser).
- With an empty support every iteration equals brp_power on X, also with a
  new A1 per iteration (the draw of that iteration).
- Planted mistakes are caught.
"""
import inspect

import numpy as np
import pytest

from oracle import completion_ref as c
from oracle import godec_ref as g


def _case(m=120, n=100, r=3, frac=0.3, seed=3):
    rng = np.random.default_rng(seed)
    X0 = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    miss = np.sort(rng.choice(m * n, size=int(frac * m * n), replace=False))
    X = X0.copy()
    X.flat[miss] = 0.0
    A1 = np.random.default_rng(seed + 1).standard_normal((n, r))
    return X0, X, miss, A1


@pytest.mark.parametrize("q", [0, 1, 2])
def test_exact_recovery(q):
    X0, X, miss, A1 = _case()
    tr = c.godec_completion(X, 3, q, A1, miss, 100)
    assert np.linalg.norm(tr.L - X0) / np.linalg.norm(X0) <= 1e-12
    assert tr.rel_err_sq[-1] <= 1e-24


def test_imputation_invariant_and_s_step():
    X0, X, miss, A1 = _case(seed=5)
    tr = c.godec_completion(X, 3, 1, A1, miss, 3)
    D = X - tr.S
    obs = np.ones(X.size, bool)
    obs[miss] = False
    assert np.array_equal(D.flat[obs], X.flat[obs])
    assert np.max(np.abs(D.flat[miss] - tr.L.flat[miss])) <= 1e-12 * np.max(np.abs(X))
    E = X - tr.L - tr.S
    assert np.all(E.flat[miss] == 0.0)


def test_empty_support_is_plain_brp():
    X0, X, _, A1 = _case(seed=7)
    X = X + 0.1 * np.random.default_rng(8).standard_normal(X.shape)
    tr = c.godec_completion(X, 3, 1, A1, np.zeros(0, np.int64), 4)
    ref = g.brp_power(X, A1, 1)
    assert np.linalg.norm(tr.L - ref.L) <= 1e-12 * np.linalg.norm(ref.L)
    assert not tr.S.any()


@pytest.mark.parametrize("iters", [1, 3])
def test_empty_support_redrawn_a1_uses_the_iterations_draw(iters):
    """With an empty support S stays 0, so with a new A1 per iteration the
    last iteration's L is brp_power on X with the last draw, A1(iters - 1);
    with q = 0 on a noisy X that L depends on A1, so another iteration's
    draw gives another L."""
    _, X, _, _ = _case(seed=9)
    X = X + 0.1 * np.random.default_rng(10).standard_normal(X.shape)
    draw = lambda t: np.random.default_rng(50 + t).standard_normal((X.shape[1], 3))
    tr = c.godec_completion(X, 3, 0, draw, np.zeros(0, np.int64), iters)
    ref = g.brp_power(X, draw(iters - 1), 0)
    assert np.linalg.norm(tr.L - ref.L) <= 1e-12 * np.linalg.norm(ref.L)
    other = g.brp_power(X, draw(iters), 0)
    assert np.linalg.norm(tr.L - other.L) > 1e-6 * np.linalg.norm(ref.L)


def _mutant(func, old, new):
    fsrc = inspect.getsource(func)
    assert old in fsrc
    msrc = inspect.getsource(c)
    ns = {"__name__": "oracle.completion_mutant", "__package__": "oracle"}
    exec(compile(msrc.replace(fsrc, fsrc.replace(old, new, 1)), "<mutant>", "exec"), ns)
    return ns


def _recovers(ns):
    X0, X, miss, A1 = _case()
    try:
        tr = ns["godec_completion"](X, 3, 1, A1, miss, 100)
    except Exception:
        return False
    return np.linalg.norm(tr.L - X0) / np.linalg.norm(X0) <= 1e-12


@pytest.mark.parametrize("func,old,new", [
    (c.fixed_support_step, "S.flat[support] = R.flat[support]", "S.flat[support] = -R.flat[support]"),
    (c.godec_completion, "res = godec_ref.brp_power(X - S, A, q, rank_tol)",
     "res = godec_ref.brp_power(X + S, A, q, rank_tol)"),
    (c.godec_completion, "R = X - res.L", "R = X - res.L.T.T * 0.5"),
])
def test_planted_mistake_is_caught(func, old, new):
    assert _recovers(dict(vars(c)))
    assert not _recovers(_mutant(func, old, new))
