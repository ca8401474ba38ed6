"""Pins for the oracle's low-rank step (Algorithm 1 L-update, Eq. 5-9)."""
import numpy as np
import pytest

from oracle import godec_ref as g


def _rank_r(m, n, r, seed, spread=0.6):
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((m, r)))[0]
    V = np.linalg.qr(rng.standard_normal((n, r)))[0]
    s = 10.0 * spread ** np.arange(r)
    return (U * s) @ V.T


@pytest.mark.parametrize("q", [0, 1, 2, 3])
@pytest.mark.parametrize("shape", [(60, 40), (40, 60), (33, 33)])
def test_exact_rank_r_reproduced(q, shape):
    """P1: on a rank-r input with S = 0 and no noise BRP returns X itself."""
    m, n = shape
    X = _rank_r(m, n, 5, seed=m * 7 + q, spread=0.8)
    A1 = np.random.default_rng(q).standard_normal((n, 5))
    res = g.brp_power(X, A1, q)
    assert res.r_eff == 5
    assert g.rel_fro(res.L, X) < 1e-12
    assert np.linalg.matrix_rank(res.L, tol=1e-10 * np.linalg.norm(X, 2)) == 5


@pytest.mark.parametrize("q", [0, 1, 2])
def test_rank_drop_restarts_with_smaller_rank(q):
    """Alg. 1 rank check: exact rank 3 with r = 5 is detected; L = X."""
    X = _rank_r(50, 40, 3, seed=11 + q)
    A1 = np.random.default_rng(5).standard_normal((40, 5))
    res = g.brp_power(X, A1, q)
    assert res.r_eff == 3
    assert g.rel_fro(res.L, X) < 1e-12


def test_rank_zero_input():
    res = g.brp_power(np.zeros((10, 8)), np.ones((8, 2)), 1)
    assert res.r_eff == 0 and not res.L.any()


@pytest.mark.parametrize("q", [1, 2])
def test_matches_truncated_svd_on_large_gap(q):
    """P3: with lambda_{r+1}/lambda_r = 1e-3 the BRP approximation equals
    LAPACK's truncated SVD up to (gap)^(2p)-size terms."""
    rng = np.random.default_rng(3)
    m, n, r = 80, 50, 4
    U = np.linalg.qr(rng.standard_normal((m, n)))[0]
    V = np.linalg.qr(rng.standard_normal((n, n)))[0]
    s = np.concatenate([[9, 7, 5, 3], 3e-3 * 0.9 ** np.arange(n - r)])
    X = (U * s) @ V.T
    A1 = rng.standard_normal((n, r))
    res = g.brp_power(X, A1, q)
    Lsvd = g.truncated_svd(X, r)
    assert g.rel_fro(res.L, Lsvd) < 1e-9


def test_theorem3_bound_q0_every_draw():
    """P6: Theorem 3 (Appendix II) bounds ||X - L||^2 for every draw of A1
    for the q = 0 step with the A2 = Y1 update."""
    rng = np.random.default_rng(5)
    for _ in range(60):
        m, n, r = 50, 30, 3
        X = rng.standard_normal((m, n)) @ np.diag(0.75 ** np.arange(n)) \
            @ rng.standard_normal((n, n))
        U, lam, Vt = np.linalg.svd(X, full_matrices=False)
        V = Vt.T
        A1 = rng.standard_normal((n, r))
        L = g.brp_power(X, A1, 0, rank_tol=0.0).L
        err = np.linalg.norm(X - L, 2) ** 2
        L1, L2 = np.diag(lam[:r]), np.diag(lam[r:])
        V1, V2 = V[:, :r], V[:, r:]
        bound = np.linalg.norm(L2 @ L2 @ (V2.T @ A1) @ np.linalg.pinv(V1.T @ A1)
                               @ np.linalg.inv(L1), 2) ** 2 \
            + np.linalg.norm(L2, 2) ** 2
        assert err <= bound * (1 + 1e-10)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_invariant_under_a1_times_invertible(q):
    """P7: L depends on A1 only through range(A1)."""
    rng = np.random.default_rng(9)
    X = rng.standard_normal((70, 45))
    A1 = rng.standard_normal((45, 6))
    T = rng.standard_normal((6, 6)) + 3 * np.eye(6)
    a = g.brp_power(X, A1, q).L
    b = g.brp_power(X, A1 @ T, q).L
    assert g.rel_fro(a, b) < 1e-11


def test_q0_is_eq5_closed_form():
    """At q = 0 Algorithm 1 is Eq. 5 with A2 = X A1 and A1 <- X^T A2."""
    rng = np.random.default_rng(2)
    X = rng.standard_normal((40, 30))
    A1 = rng.standard_normal((30, 4))
    Y1 = X @ A1
    A2 = Y1
    Y2 = X.T @ A2
    Y1n = X @ Y2
    L = Y1n @ np.linalg.solve(A2.T @ Y1n, Y2.T)
    assert g.rel_fro(g.brp_power(X, A1, 0).L, L) < 1e-12


def test_power_scheme_improves_error_on_slow_decay():
    """Sec. 3.1.2: the error decreases as q grows on a slowly decaying
    spectrum (checked on average over draws)."""
    rng = np.random.default_rng(4)
    m, n, r = 120, 80, 5
    U = np.linalg.qr(rng.standard_normal((m, n)))[0]
    V = np.linalg.qr(rng.standard_normal((n, n)))[0]
    X = (U * 0.97 ** np.arange(n)) @ V.T
    errs = []
    for q in (0, 1, 2):
        e = [np.linalg.norm(X - g.brp_power(
            X, rng.standard_normal((n, r)), q).L) for _ in range(10)]
        errs.append(np.mean(e))
    assert errs[0] > errs[1] > errs[2]


def test_factor_frobenius_identity():
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal((30, 3)), rng.standard_normal((20, 3))
    c, d = rng.standard_normal((30, 3)), rng.standard_normal((20, 3))
    ref = np.linalg.norm(a @ b.T - c @ d.T) / np.linalg.norm(c @ d.T)
    assert abs(g.rel_fro_factors(a, b, c, d) - ref) < 1e-7


@pytest.mark.parametrize("q", [0, 1, 2])
def test_literal_lines_agree_where_accurate(q):
    """P2: the literal evaluation of Algorithm 1's lines and the restated
    evaluation agree on a well-conditioned low-rank + sparse input."""
    from paper_1309_0302_amd import workloads as wl
    w = wl.tiny(300, 200, 5, seed=3)
    A1 = np.random.default_rng(q).standard_normal((200, 5))
    a = g.brp_power(w.X, A1, q)
    b = g.brp_power_literal(w.X, A1, q)
    assert a.r_eff == b.r_eff == 5
    assert g.rel_fro(a.L, b.L) < 1e-12
    # A2^T Y1 = Y2^T Y2 = R2^T R2: same singular values of C both ways
    assert np.allclose(a.sing_c, b.sing_c, rtol=1e-9)
    # the core's singular values (the L~ scale) agree as well
    assert np.allclose(a.sing_core, b.sing_core, rtol=1e-9) if q > 0 else True


def test_literal_lines_lose_digits_on_graded_spectrum():
    """Why the restated form is the oracle: on a rank-5 input with
    lambda_5/lambda_1 = 0.13 the literal products are graded like
    lambda^{3p} and lose accuracy at q = 2; the restated form does not."""
    X = _rank_r(60, 40, 5, seed=7)
    A1 = np.random.default_rng(0).standard_normal((40, 5))
    assert g.rel_fro(g.brp_power(X, A1, 2, rank_tol=0.0).L, X) < 1e-12
    assert g.rel_fro(g.brp_power_literal(X, A1, 2, rank_tol=0.0).L, X) > 1e-9


def test_default_rank_rule_is_on_the_scale_of_c():
    """Reading R5: the default tolerance r*2^-52 applies to C = A2^T Y1, whose
    singular values scale like lambda^{4p}.  At q = 2 a component with
    lambda_5/lambda_1 = 0.13 falls below it and the rank drops to 4; at q = 0
    it is kept."""
    X = _rank_r(60, 40, 5, seed=7)
    A1 = np.random.default_rng(0).standard_normal((40, 5))
    assert g.brp_power(X, A1, 2).r_eff == 4
    assert g.brp_power_literal(X, A1, 2).r_eff == 4
    assert g.brp_power(X, A1, 0).r_eff == 5


def test_rank_zero_carry_gives_zero_L():
    """After a rank drop to 0 the next steps run with no column of A1 (reading
    R5): L = 0, and the loop keeps S = the top-k of X."""
    D = np.zeros((30, 20))
    A1 = np.random.default_rng(0).standard_normal((20, 3))
    res = g.brp_power(D, A1, 1)
    assert res.r_eff == 0 and not res.L.any()
    res0 = g.brp_power(D, A1[:, :0], 1)
    assert res0.r_eff == 0 and res0.L.shape == (30, 20) and not res0.L.any()
    lit = g.brp_power_literal(D, A1[:, :0], 2)
    assert lit.r_eff == 0 and not lit.L.any()


@pytest.mark.parametrize("q", [1, 2])
def test_theorem4_bound_projection_form_every_draw(q):
    """App. II, Thm. 4: for the power scheme, ||X - L||^2 <=
    (||L2^{2p} (V2^T A1)(V1^T A1)^+ L1^{-p}||^2 + ||L2^p||^2)^{1/p}, p = 2q+1,
    for every draw of A1, with L = X P_{Y2} (spectral norm).  The bound is
    tight on these inputs (ratios up to 0.9999), so a wrong power, a
    transposed operand or a missing re-orthonormalisation breaks it."""
    rng = np.random.default_rng(5 + q)
    p = 2 * q + 1
    worst = 0.0
    for _ in range(100):
        m, n, r = 50, 30, 3
        X = rng.standard_normal((m, n)) @ np.diag(0.75 ** np.arange(n)) \
            @ rng.standard_normal((n, n))
        U, lam, Vt = np.linalg.svd(X, full_matrices=False)
        V = Vt.T
        A1 = rng.standard_normal((n, r))
        L = g.brp_projection(X, A1, q).L
        err = np.linalg.norm(X - L, 2) ** 2
        L1, L2 = np.diag(lam[:r]), np.diag(lam[r:])
        V1, V2 = V[:, :r], V[:, r:]
        t1 = np.linalg.norm(np.linalg.matrix_power(L2, 2 * p) @ (V2.T @ A1)
                            @ np.linalg.pinv(V1.T @ A1)
                            @ np.linalg.matrix_power(np.linalg.inv(L1), p), 2) ** 2
        t2 = np.linalg.norm(np.linalg.matrix_power(L2, p), 2) ** 2
        bound = (t1 + t2) ** (1.0 / p)
        assert err <= bound * (1 + 1e-10)
        worst = max(worst, err / bound)
    assert worst > 0.5          # the bound is not vacuous here


def test_projection_equals_root_form_at_q0():
    rng = np.random.default_rng(11)
    X = rng.standard_normal((40, 30)) @ np.diag(0.8 ** np.arange(30)) @ rng.standard_normal((30, 30))
    A1 = rng.standard_normal((30, 4))
    a = g.brp_projection(X, A1, 0).L
    b = g.brp_power(X, A1, 0).L
    assert g.rel_fro(a, b) < 1e-12


@pytest.mark.parametrize("q", [0, 1, 2])
def test_projection_reproduces_rank_r(q):
    rng = np.random.default_rng(12 + q)
    X = rng.standard_normal((60, 4)) @ rng.standard_normal((4, 45))
    L = g.brp_projection(X, rng.standard_normal((45, 4)), q).L
    assert g.rel_fro(L, X) < 1e-12


def test_projection_loop_recovers_w1_like_problem():
    """GoDec with the projection L step on a planted low-rank + sparse X
    recovers the low-rank part (the same fixed point as the root form)."""
    rng = np.random.default_rng(13)
    m, n, r, k = 200, 150, 4, 1500
    L0 = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    X = L0.copy()
    idx = rng.choice(m * n, size=k, replace=False)
    X.flat[idx] += rng.uniform(-10, 10, size=k)
    A1 = rng.standard_normal((n, r))
    tr = g.godec_brp(X, r, k, 1, A1, 30, lstep="proj")
    assert g.rel_fro(tr.L, L0) < 1e-8
    ref = g.godec_brp(X, r, k, 1, A1, 30)
    assert g.rel_fro(tr.L, ref.L) < 1e-8


@pytest.mark.parametrize("q", [0, 1])
def test_warm_start_reaches_the_same_fixed_point(q):
    """Warm-started chains (the previous right factor in place of A1) reach
    the planted low-rank part, as the cold-started loop does, and never
    fewer digits of it."""
    rng = np.random.default_rng(21 + q)
    m, n, r, k = 200, 150, 4, 1500
    L0 = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    X = L0.copy()
    idx = rng.choice(m * n, size=k, replace=False)
    X.flat[idx] += rng.uniform(-10, 10, size=k)
    A1 = rng.standard_normal((n, r))
    warm = g.godec_brp(X, r, k, q, A1, 40, warm=True)
    cold = g.godec_brp(X, r, k, q, A1, 40)
    assert g.rel_fro(warm.L, L0) < 1e-8
    assert g.rel_fro(warm.L, L0) <= max(10 * g.rel_fro(cold.L, L0), 1e-12)


def test_warm_start_first_iteration_is_the_cold_one():
    rng = np.random.default_rng(23)
    X = rng.standard_normal((80, 60))
    A1 = rng.standard_normal((60, 3))
    a = g.godec_brp(X, 3, 100, 1, A1, 1, warm=True)
    b = g.godec_brp(X, 3, 100, 1, A1, 1)
    assert np.array_equal(a.L, b.L)

