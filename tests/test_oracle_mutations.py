"""Planted mistakes in the oracle must be caught by its pins.

Each case rewrites one token of an oracle function's source (a dropped term,
a wrong exponent, a transposed operand, a flipped tie-break), executes the
mutant in a copy of the module namespace and checks that at least one pin
fails on it while the unmutated function passes.  Runs on the CPU only.
"""
import inspect
import textwrap

import numpy as np
import pytest

from oracle import godec_ref as g


def mutant(func, old, new):
    src = textwrap.dedent(inspect.getsource(func))
    assert old in src, f"mutation anchor {old!r} not found"
    ns = dict(vars(g))
    exec(compile(src.replace(old, new, 1), "<mutant>", "exec"), ns)
    return ns[func.__name__], ns


def _rank_r(m, n, r, seed):
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((m, r)))[0]
    V = np.linalg.qr(rng.standard_normal((n, r)))[0]
    return (U * (10.0 * 0.8 ** np.arange(r))) @ V.T


def pin_exact_rank(brp):
    """Max error of BRP on exact rank-r inputs over shapes and powers."""
    worst = 0.0
    for (m, n) in ((50, 40), (40, 50), (30, 30)):
        for q in (0, 1, 2):
            X = _rank_r(m, n, 4, seed=m + n + q)
            A1 = np.random.default_rng(q).standard_normal((n, 4))
            try:
                L = brp(X, A1, q).L
                worst = max(worst, g.rel_fro(L, X))
            except Exception:
                return np.inf
    return worst


def pin_svd_gap(brp):
    rng = np.random.default_rng(3)
    m, n, r = 60, 40, 3
    U = np.linalg.qr(rng.standard_normal((m, n)))[0]
    V = np.linalg.qr(rng.standard_normal((n, n)))[0]
    s = np.concatenate([[9, 6, 4], 4e-3 * 0.9 ** np.arange(n - r)])
    X = (U * s) @ V.T
    try:
        return max(g.rel_fro(brp(X, rng.standard_normal((n, r)), q).L,
                             g.truncated_svd(X, r)) for q in (1, 2))
    except Exception:
        return np.inf


def pin_literal(brp):
    """Agreement with the literal lines on a moderately conditioned input."""
    from paper_1309_0302_amd import workloads as wl
    w = wl.tiny(120, 80, 4, seed=3)
    worst = 0.0
    for q in (0, 1, 2):
        A1 = np.random.default_rng(q).standard_normal((80, 4))
        try:
            worst = max(worst, g.rel_fro(brp(w.X, A1, q).L,
                                         g.brp_power_literal(w.X, A1, q).L))
        except Exception:
            return np.inf
    return worst


BRP_MUTANTS = [
    ("root exponent 1/(2q)", "root = s ** (1.0 / p)", "root = s ** (1.0 / max(p - 1, 1))"),
    ("power count p-1", "for _ in range(p):", "for _ in range(max(p - 1, 1)):"),
    ("transposed Gram product", "np.linalg.qr(D.T @ (D @ Z))", "np.linalg.qr(D @ (D.T @ Z[:D.shape[0]]) if D.shape[0] == D.shape[1] else D.T @ (D @ Z))"),
    ("B chain without L~ power", "B = ltilde_apply(D, Q2, q)", "B = D @ Q2"),
    ("right factor not rotated", "right = Q2 @ Vt.T", "right = Q2"),
    ("left factor missing U", "left = Q1 @ (U * root)", "left = Q1 * root"),
]


@pytest.mark.parametrize("name,old,new", BRP_MUTANTS, ids=[m[0] for m in BRP_MUTANTS])
def test_brp_mutants_caught(name, old, new):
    assert pin_exact_rank(g.brp_power) < 1e-12 and pin_svd_gap(g.brp_power) < 1e-8
    assert pin_literal(g.brp_power) < 1e-8
    bad, _ = mutant(g.brp_power, old, new)
    assert (pin_exact_rank(bad) > 1e-6 or pin_svd_gap(bad) > 1e-6
            or pin_literal(bad) > 1e-5), name


def brute(R, k):
    a = np.abs(R).ravel()
    order = sorted(range(a.size), key=lambda i: (-a[i], i))
    return np.array(sorted(i for i in order[:k] if a[i] != 0), dtype=np.int64)


def pin_topk(ht):
    rng = np.random.default_rng(0)
    for _ in range(6):
        R = rng.integers(-3, 4, size=(6, 7)).astype(float)
        for k in range(0, 44, 3):
            try:
                idx, _ = ht(R, k)
            except Exception:
                return False
            if not np.array_equal(np.asarray(idx), brute(R, k)):
                return False
    return True


TOPK_MUTANTS = [
    ("ties by descending index", "take = k - above.size", "ties = ties[::-1]; take = k - above.size"),
    ("off-by-one k", "np.partition(a, N - k)[N - k]", "np.partition(a, N - k + 1)[N - k + 1] if k > 1 else np.partition(a, N - k)[N - k]"),
    ("zeros kept", "if t == 0:", "if False:"),
    (">= instead of >", "above = np.flatnonzero(a > t)", "above = np.flatnonzero(a >= t)"),
]


@pytest.mark.parametrize("name,old,new", TOPK_MUTANTS, ids=[m[0] for m in TOPK_MUTANTS])
def test_topk_mutants_caught(name, old, new):
    assert pin_topk(g.hard_threshold)
    bad, _ = mutant(g.hard_threshold, old, new)
    assert not pin_topk(bad), name


LOOP_MUTANTS = [
    ("sign flip in residual", "R = X - L", "R = X + L"),
    ("D not updated from S", "D = X - S", "D = X"),
]


@pytest.mark.parametrize("name,old,new", LOOP_MUTANTS, ids=[m[0] for m in LOOP_MUTANTS])
def test_loop_mutants_caught(name, old, new):
    from paper_1309_0302_amd import workloads as wl
    w = wl.tiny(60, 50, 3, rho=0.03, amp=5.0, noise_std=0.0, seed=4)
    A1 = np.random.default_rng(1).standard_normal((50, 3))
    ref = g.godec_naive(w.X, 3, w.k, 25)
    good = g.godec_brp(w.X, 3, w.k, 1, A1, 25)
    assert g.rel_fro(good.L, ref.L) < 1e-9
    bad, _ = mutant(g.godec_brp, old, new)
    tb = bad(w.X, 3, w.k, 1, A1, 25)
    assert g.rel_fro(tb.L, ref.L) > 1e-6, name
