"""Pins of the GreBsmo oracle (Sec. 3.2.1) against things other than itself.

- Eq. 12's soft threshold is the minimiser of a scalar objective: checked by
  brute-force grid search, and on hand-worked values.
- The QR form of the inner iteration (Eq. 13) must give the same U V and S
  as the alternating least-squares rules with pseudo-inverses (Eq. 11).
- The S update satisfies the optimality (KKT) conditions of the l1 problem.
- Every update is a block minimisation, so F = 1/2 ||X - U V - S||^2 +
  lambda ||S||_1 never increases (within and across rank stages).
- With a spectral gap and enough power steps, the greedy directions span the
  top right singular vectors (LAPACK SVD).
- With lambda so large that S stays 0, GreBsmo is subspace iteration and
  reaches the truncated SVD (LAPACK).
- A planted low-rank + sparse matrix is recovered within the rel. err. 1e-2
  success criterion of Sec. 5.4.
- Planted mistakes in the oracle (a wrong threshold, a transposed operand, a
  dropped S) make at least one of these pins fail.
CPU only.
"""
import inspect

import numpy as np
import pytest

from oracle import grebsmo_ref as g
from paper_1309_0302_amd import workloads as wl


def test_soft_threshold_hand_values():
    R = np.array([3.0, -0.5, 1.0, -2.0, 0.0, 1.25])
    got = g.soft_threshold(R, 1.0)
    assert np.array_equal(got, np.array([2.0, 0.0, 0.0, -1.0, 0.0, 0.25]))


def test_soft_threshold_minimises_scalar_objective():
    rng = np.random.default_rng(0)
    grid = np.linspace(-8.0, 8.0, 160001)       # step 1e-4
    for _ in range(40):
        r = rng.uniform(-6, 6)
        lam = rng.uniform(0.0, 3.0)
        f = 0.5 * (r - grid) ** 2 + lam * np.abs(grid)
        best = grid[np.argmin(f)]
        assert abs(g.soft_threshold(np.array([r]), lam)[0] - best) <= 1.5e-4


def _problem(m, n, r, seed, rho=0.05, amp=5.0):
    X, L0, _ = wl.planted_pm(m, n, r, rho=rho, amp=amp, seed=seed)
    return X + 1e-2 * np.random.default_rng(seed + 1).standard_normal((m, n)), L0


def test_inner_step_equals_als_rules():
    X, _ = _problem(40, 30, 3, 1)
    rng = np.random.default_rng(2)
    S = g.soft_threshold(X, 2.0)
    V = rng.standard_normal((4, 30))
    U1, V1, S1 = g.inner_step(X, S, V, 0.3)
    U2, V2, S2 = g.inner_step_als(X, S, V, 0.3)
    L1, L2 = U1 @ V1, U2 @ V2
    assert np.linalg.norm(L1 - L2) <= 1e-10 * np.linalg.norm(L2)
    assert np.max(np.abs(S1 - S2)) <= 1e-10
    # U is orthonormal in the QR form
    assert np.allclose(U1.T @ U1, np.eye(4), atol=1e-12)


def test_s_update_kkt():
    X, _ = _problem(50, 40, 3, 3)
    lam = 0.4
    res = g.grebsmo(X, 3, 1, 3, lam, 2, np.random.default_rng(4).standard_normal((40, 3)))
    E = X - res.U @ res.V - res.S
    on = res.S != 0
    assert on.any() and (~on).any()
    assert np.max(np.abs(E[on] - lam * np.sign(res.S[on]))) <= 1e-12
    assert np.max(np.abs(E[~on])) <= lam + 1e-12


def test_objective_never_increases():
    X, _ = _problem(100, 80, 4, 5)
    res = g.grebsmo(X, 4, 1, 5, 0.2, 2, np.random.default_rng(6).standard_normal((80, 4)),
                    track=True)
    F = np.array(res.objective)
    assert len(F) == 20
    assert np.all(np.diff(F) <= 1e-10 * F[0])
    assert res.ranks == [1, 2, 3, 4]


def _gapped(m, n, top, seed):
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((m, n)))[0]
    V = np.linalg.qr(rng.standard_normal((n, n)))[0]
    s = np.concatenate([top, 1e-2 * 0.9 ** np.arange(n - len(top))])
    return (U * s) @ V.T, V


def test_greedy_directions_span_top_right_singular_vectors():
    X, V = _gapped(70, 50, [10.0, 8.0, 6.0], 7)
    Om = np.random.default_rng(8).standard_normal((50, 3))
    Z = g.greedy_directions(X, Om, 6)
    assert Z.shape == (3, 50)
    P1 = Z.T @ Z
    P2 = V[:, :3] @ V[:, :3].T
    assert np.linalg.norm(P1 - P2) <= 1e-8


def _greedy_capture(X, res, lam):
    """Fraction of the top-dr singular energy of dF/dV = X - U V - S (from
    the previous stage's state, by LAPACK SVD) that each later stage's
    appended rows capture (1 = the top right singular subspace, Eq. 14)."""
    worst = 1.0
    for s in range(1, len(res.added)):
        U, V, S = res.states[s - 1]
        R = X - U @ V - S
        Z = res.added[s]
        sv = np.linalg.svd(R, compute_uv=False)
        got = np.linalg.norm(R @ Z.T) ** 2
        worst = min(worst, got / np.sum(sv[:Z.shape[0]] ** 2))
    return worst


def test_greedy_rows_are_top_singular_directions_of_the_derivative():
    X, _ = _problem(90, 70, 3, 14)
    res = g.grebsmo(X, 3, 1, 4, 0.3, 100, np.random.default_rng(15).standard_normal((70, 3)),
                    track=True)
    assert len(res.added) == 3
    assert _greedy_capture(X, res, 0.3) >= 1.0 - 1e-9


def test_power_must_be_positive():
    with pytest.raises(ValueError):
        g.greedy_directions(np.eye(3), np.ones((3, 1)), 0)


@pytest.mark.parametrize("dr", [1, 3])
def test_huge_lambda_gives_truncated_svd(dr):
    X, _ = _gapped(60, 40, [9.0, 7.0, 5.0], 9)
    Om = np.random.default_rng(10).standard_normal((40, 3))
    res = g.grebsmo(X, 3, dr, 60, 1e6, 2, Om)
    assert not res.S.any()
    U, s, Vt = np.linalg.svd(X)
    Lsvd = (U[:, :3] * s[:3]) @ Vt[:3]
    assert np.linalg.norm(res.U @ res.V - Lsvd) <= 1e-9 * np.linalg.norm(Lsvd)


def test_planted_recovery_g1():
    w = wl.g1()
    Om = np.random.default_rng(11).standard_normal((500, w.r))
    res = g.grebsmo(w.X, w.r, w.dr, w.K, w.lam, w.power, Om)
    L = res.U @ res.V
    assert np.linalg.norm(L - w.L0) / np.linalg.norm(w.L0) <= 1e-2
    assert res.ranks[-1] == w.r


def test_tau_stops_early():
    X, _ = _problem(60, 50, 2, 12)
    Om = np.random.default_rng(13).standard_normal((50, 6))
    full = g.grebsmo(X, 6, 1, 5, 0.2, 2, Om)
    tau = full.rel_err[2] * 1.0000001
    short = g.grebsmo(X, 6, 1, 5, 0.2, 2, Om, tau=tau)
    assert len(short.rel_err) <= 3
    assert short.rel_err[-1] <= tau


# ---- planted mistakes ---------------------------------------------------------

def _mutant(func, old, new):
    """Namespace of the whole oracle module re-executed with one token of
    ``func`` changed (so every caller of ``func`` sees the mutant)."""
    fsrc = inspect.getsource(func)
    assert old in fsrc, f"mutation anchor {old!r} not found"
    msrc = inspect.getsource(g)
    assert msrc.count(fsrc) == 1
    ns = {"__name__": "oracle_mutant"}
    exec(compile(msrc.replace(fsrc, fsrc.replace(old, new, 1)), "<mutant>", "exec"), ns)
    return ns


def _pins_pass(ns) -> bool:
    """Runs the pins above against the functions of namespace ns."""
    soft, inner, greedy, run = ns["soft_threshold"], ns["inner_step"], \
        ns["greedy_directions"], ns["grebsmo"]
    try:
        # soft threshold minimises the scalar objective
        grid = np.linspace(-8.0, 8.0, 16001)
        for r, lam in ((3.0, 1.0), (-2.5, 0.7), (0.3, 0.5)):
            best = grid[np.argmin(0.5 * (r - grid) ** 2 + lam * np.abs(grid))]
            if abs(soft(np.array([r]), lam)[0] - best) > 2e-3:
                return False
        # QR form equals the ALS rules
        X, _ = _problem(40, 30, 3, 1)
        S = g.soft_threshold(X, 2.0)
        V = np.random.default_rng(2).standard_normal((4, 30))
        U1, V1, S1 = inner(X, S, V, 0.3)
        U2, V2, S2 = g.inner_step_als(X, S, V, 0.3)
        if np.linalg.norm(U1 @ V1 - U2 @ V2) > 1e-8 * np.linalg.norm(U2 @ V2):
            return False
        if np.max(np.abs(S1 - S2)) > 1e-8:
            return False
        # greedy directions
        Xg, Vg = _gapped(70, 50, [10.0, 8.0, 6.0], 7)
        Z = greedy(Xg, np.random.default_rng(8).standard_normal((50, 3)), 6)
        if np.linalg.norm(Z.T @ Z - Vg[:, :3] @ Vg[:, :3].T) > 1e-6:
            return False
        # objective monotone and KKT
        X, _ = _problem(100, 80, 4, 5)
        res = run(X, 4, 1, 5, 0.2, 2, np.random.default_rng(6).standard_normal((80, 4)),
                  track=True)
        F = np.array(res.objective)
        if not np.all(np.diff(F) <= 1e-10 * F[0]):
            return False
        E = X - res.U @ res.V - res.S
        on = res.S != 0
        if np.max(np.abs(E[on] - 0.2 * np.sign(res.S[on])), initial=0) > 1e-9:
            return False
        if np.max(np.abs(E[~on]), initial=0) > 0.2 + 1e-9:
            return False
        # greedy rows follow the derivative
        X, _ = _problem(90, 70, 3, 14)
        res = run(X, 3, 1, 4, 0.3, 100,
                  np.random.default_rng(15).standard_normal((70, 3)), track=True)
        if _greedy_capture(X, res, 0.3) < 1.0 - 1e-9:
            return False
    except Exception:
        return False
    return True


def test_unmutated_oracle_passes_the_pins():
    assert _pins_pass(dict(vars(g)))


@pytest.mark.parametrize("func,old,new", [
    (g.soft_threshold, "np.abs(R) - lam", "np.abs(R) - lam / 2"),      # threshold scale
    (g.soft_threshold, "np.sign(R) *", "-np.sign(R) *"),              # sign
    (g.inner_step, "orth(D @ V.T)", "orth(X @ V.T)"),                 # dropped S
    (g.inner_step, "V = U.T @ D", "V = U.T @ X"),                     # dropped S
    (g.inner_step, "X - U @ V, lam", "X - S - U @ V, lam"),           # S counted twice
    (g.greedy_directions, "orth(R.T @ (R @ Z))", "orth(R.T @ Z[:R.shape[0]])"),
    (g.grebsmo_stage, "R = X - U @ V - S", "R = X - U @ V"),           # dropped S in dF/dV
])
def test_planted_mistake_is_caught(func, old, new):
    ns = _mutant(func, old, new)
    assert not _pins_pass(ns)
