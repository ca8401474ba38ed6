"""FP64 oracle of GoDec by bilateral random projection (test infrastructure).

Zhou & Tao, "Unmixing Incoherent Structures of Big Data by Randomized or
Greedy Decomposition", arXiv 1309.0302.  Everything here is plain NumPy /
LAPACK in float64, written to be read against the paper, not to be fast.
Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
it; the GPU library never does.

Notation follows the paper: X is m x n, r the rank bound, k the cardinality
bound, q the power, p = 2q + 1, S_t the sparse part after iteration t and
D = X - S_{t-1}.

Readings of the paper (where it is silent or ambiguous) used here:

R1  The loop test of Algorithm 1 is evaluated after each iteration (with
    L_0 = X and S_0 = 0 it would be false before the first one), and the
    workloads fix the iteration count T instead of a tolerance.
R2  By default A1 is drawn once and kept for all iterations (R15 covers a
    redrawn A1); Algorithm 1 then builds A2 from Y1 as Sec. 3.1.1 describes,
    so no independent A2 is used.
R3  The operator L~ = [(X - S)(X - S)^T]^q (X - S) is never formed: L~ Z is
    evaluated right to left as a chain of products with D and D^T, which is
    the same matrix product by associativity.
R4  The fractional power [.]^{1/(2q+1)} of the non-symmetric r x r core is
    taken through its SVD (the paper budgets "an SVD of an r x r matrix"
    for it): U diag(s^{1/p}) V^T.
R5  rank(A2^T Y1) is the numerical rank of the r x r matrix C = A2^T Y1.
    Because A2 = Y1 (before the update) and Y2 = L~^T A2, C = Y2^T Y2 holds
    exactly, so its singular values are the squares of those of Y2; they
    are computed from Y2 (whose small singular values LAPACK resolves to
    working precision, unlike those of the product C) and compared with the
    MATLAB ``rank`` default, tol = r * 2^-52 * s_1(C).  When the rank drops
    to r' < r the step restarts with the first r' columns of A1 ("go to the
    first step"), and r stays r' for the following iterations.
R6  The hard threshold keeps the k entries of |X - L| that come first in the
    order (|value| descending, row-major linear index ascending), minus any
    exact zeros (Eq. 4 and Algorithm 1 ask for the nonzero subset).
R7  The paper's relative error is the squared ratio ||X - L - S||_F^2 /
    ||X||_F^2 (Sec. 5); both it and its square root are reported.
R8  L is evaluated through exact identities of Algorithm 1's lines
    (A2^T Y1 = R2^T R2 and the R factor of Y1 = L~ Y2) instead of forming the
    graded products Y1, Y2 literally; see ``brp_power``.  The literal lines
    are kept in ``brp_power_literal`` and pin it where they are accurate.
R15 With a redrawn A1 (an option of the library; the MSE training of
    Algorithm 4 draws a new A1 every iteration), iteration t uses the first
    r' columns of its own draw A1(t), r' being the rank kept after the
    earlier iterations (R5).
"""

from dataclasses import dataclass, field

import time

import numpy as np

RANK_TOL_DEFAULT_ULP = 2.0 ** -52


# ---------------------------------------------------------------------------
# The operator L~ of Algorithm 1 (its definition line), applied to a panel.
# ---------------------------------------------------------------------------

def ltilde_apply(D: np.ndarray, Z: np.ndarray, q: int) -> np.ndarray:
    """Return L~ Z with L~ = (D D^T)^q D (Algorithm 1; reading R3)."""
    Y = D @ Z
    for _ in range(q):
        Y = D @ (D.T @ Y)
    return Y


def ltilde_apply_t(D: np.ndarray, W: np.ndarray, q: int) -> np.ndarray:
    """Return L~^T W = D^T (D D^T)^q W (Algorithm 1; reading R3)."""
    Y = W
    for _ in range(q):
        Y = D @ (D.T @ Y)
    return D.T @ Y


# ---------------------------------------------------------------------------
# Low-rank step: BRP with the projection update and the power scheme.
# ---------------------------------------------------------------------------

@dataclass
class BrpResult:
    L: np.ndarray            # m x n rank-(<= r) approximation
    left: np.ndarray         # m x r_eff factor, L = left @ right.T
    right: np.ndarray        # n x r_eff factor
    r_eff: int               # rank after the rank check
    sing_c: np.ndarray       # singular values of C = A2^T Y1 (via Y2), desc.
    sing_core: np.ndarray    # singular values of the core before the root


def rank_of_c(Y2: np.ndarray, rank_tol: float | None) -> tuple[int, np.ndarray]:
    """Numerical rank of C = A2^T Y1 = Y2^T Y2 (reading R5)."""
    r = Y2.shape[1]
    s_y2 = np.linalg.svd(Y2, compute_uv=False)
    s_c = s_y2 ** 2
    tol = (r * RANK_TOL_DEFAULT_ULP) if rank_tol is None else rank_tol
    if s_c[0] == 0.0:
        return 0, s_c
    return int(np.count_nonzero(s_c > tol * s_c[0])), s_c


def brp_power(D: np.ndarray, A1: np.ndarray, q: int,
              rank_tol: float | None = None) -> BrpResult:
    """One low-rank step of Algorithm 1 on D = X - S_{t-1} (Eq. 5-9).

    The algorithm's lines are
        Y1 = L~ A1, A2 = Y1;  Y2 = L~^T Y1 = Q2 R2;  Y1 = L~ Y2 = Q1 R1;
        if rank(A2^T Y1) < r: r := rank(A2^T Y1), restart;
        L = Q1 [R1 (A2^T Y1)^{-1} R2^T]^{1/(2q+1)} Q2^T.
    Evaluated literally (``brp_power_literal``) the products are graded like
    lambda^{3p} and FP64 loses about log10((lambda_1/lambda_r)^{3p}) digits.
    This function evaluates the same L through exact identities of those
    lines, so that it is accurate on any spectrum (reading R8):

    * Y2 = L~^T L~ A1 = (D^T D)^p A1.  It is built as p products with D^T D,
      each followed by a Householder QR, keeping the product of the R
      factors: Y2 = Q2 R2 exactly (rounding aside), with Q2 = the last Q.
    * A2^T Y1 = (L~^T A2)^T Y2 = Y2^T Y2 = R2^T R2, which gives the rank
      check (reading R5) and the inverse in closed form.
    * Y1 = L~ Y2 = B R2 with B = L~ Q2.  With B = Q1 R1' (QR), the R factor
      of Y1 is R1 = R1' R2, and the core becomes
      R1 (R2^T R2)^{-1} R2^T = R1' R2 R2^{-1} R2^{-T} R2^T = R1'.
    * Hence L = Q1 [R1']^{1/p} Q2^T with the root taken through the SVD of
      the r x r matrix R1' (reading R4).  At q = 0 this is Eq. 5,
      Y1 (A2^T Y1)^{-1} Y2^T.

    Pinned by: agreement with the literal lines where those are accurate;
    exact reproduction of rank-r inputs on graded spectra; LAPACK truncated
    SVD on inputs with a large spectral gap; the Theorem 3 bound at q = 0;
    invariance under A1 -> A1 T (tests/test_oracle_brp.py).
    """
    m, n = D.shape
    p = 2 * q + 1
    r = A1.shape[1]
    if r == 0:
        # an earlier rank check left no column (reading R5): L = 0
        return BrpResult(np.zeros((m, n)), np.zeros((m, 0)), np.zeros((n, 0)), 0,
                         np.zeros(0), np.zeros(0))
    while True:
        Z, R2 = np.linalg.qr(A1[:, :r])
        for _ in range(p):
            Z, Rj = np.linalg.qr(D.T @ (D @ Z))
            R2 = Rj @ R2
        Q2 = Z
        r_new, s_c = _rank_from_r2(R2, rank_tol)
        if r_new < r:
            if r_new == 0:
                return BrpResult(np.zeros((m, n)), np.zeros((m, 0)),
                                 np.zeros((n, 0)), 0, s_c, np.zeros(0))
            r = r_new          # "go to the first step" with the smaller rank
            continue
        break
    B = ltilde_apply(D, Q2, q)                  # L~ Q2 = Y1 R2^{-1}
    Q1, R1p = np.linalg.qr(B)
    U, s, Vt = np.linalg.svd(R1p)
    root = s ** (1.0 / p)
    left = Q1 @ (U * root)
    right = Q2 @ Vt.T
    return BrpResult(left @ right.T, left, right, r, s_c, s)


def brp_projection(D: np.ndarray, A1: np.ndarray, q: int) -> BrpResult:
    """The projection form of the power-scheme low-rank step: L = D P_{Y2},
    the projection of the rows of D onto range(Y2) with
    Y2 = L~^T L~ A1 = (D^T D)^p A1 — the approximation that the power-scheme
    bound of App. II (Thm. 4) analyses.  Y2 is built as p products with
    D^T D, each followed by a Householder QR (the span is unchanged), so
    L = (D Q2) Q2^T with Q2 the last Q.  At q = 0 it equals the root form
    (Eq. 5).  No rank check: it needs no inverse.

    Pinned by: the Thm. 4 deterministic bound on every draw for q = 1, 2;
    equality with brp_power at q = 0; exact reproduction of rank-r inputs
    (tests/test_oracle_brp.py).
    """
    p = 2 * q + 1
    Z, _ = np.linalg.qr(A1)
    for _ in range(p):
        Z, _ = np.linalg.qr(D.T @ (D @ Z))
    left = D @ Z
    return BrpResult(left @ Z.T, left, Z, A1.shape[1], np.zeros(0), np.zeros(0))


def _rank_from_r2(R2: np.ndarray, rank_tol: float | None):
    r = R2.shape[1]
    s_c = np.linalg.svd(R2, compute_uv=False) ** 2     # singular values of C
    tol = (r * RANK_TOL_DEFAULT_ULP) if rank_tol is None else rank_tol
    if s_c[0] == 0.0:
        return 0, s_c
    return int(np.count_nonzero(s_c > tol * s_c[0])), s_c


def brp_power_literal(D: np.ndarray, A1: np.ndarray, q: int,
                      rank_tol: float | None = None) -> BrpResult:
    """Algorithm 1's low-rank lines evaluated literally, in order.

    Accurate only while (lambda_1/lambda_r)^{3(2q+1)} stays far below 1/eps;
    used to pin ``brp_power`` on such inputs.
    """
    m, n = D.shape
    p = 2 * q + 1
    r = A1.shape[1]
    if r == 0:
        return BrpResult(np.zeros((m, n)), np.zeros((m, 0)), np.zeros((n, 0)), 0,
                         np.zeros(0), np.zeros(0))
    while True:
        A = A1[:, :r]
        Y1 = ltilde_apply(D, A, q)
        A2 = Y1
        Y2 = ltilde_apply_t(D, Y1, q)
        Y1 = ltilde_apply(D, Y2, q)
        C = A2.T @ Y1
        r_new, s_c = rank_of_c(Y2, rank_tol)
        if r_new < r:
            if r_new == 0:
                return BrpResult(np.zeros((m, n)), np.zeros((m, 0)),
                                 np.zeros((n, 0)), 0, s_c, np.zeros(0))
            r = r_new
            continue
        break
    if q == 0:
        left = Y1 @ np.linalg.inv(C)             # Eq. 5: Y1 C^{-1} Y2^T
        return BrpResult(left @ Y2.T, left, Y2, r, s_c,
                         np.linalg.svd(C, compute_uv=False))
    Q2, R2 = np.linalg.qr(Y2)
    Q1, R1 = np.linalg.qr(Y1)
    M = R1 @ np.linalg.solve(C, R2.T)            # R1 C^{-1} R2^T
    U, s, Vt = np.linalg.svd(M)
    left = Q1 @ (U * s ** (1.0 / p))
    right = Q2 @ Vt.T
    return BrpResult(left @ right.T, left, right, r, s_c, s)


# ---------------------------------------------------------------------------
# Sparse step: entry-wise hard threshold with a cardinality bound (Eq. 4).
# ---------------------------------------------------------------------------

def hard_threshold(R: np.ndarray, k: int) -> tuple[np.ndarray, np.ndarray]:
    """Support and values of S = P_Omega(R), |Omega| <= k (Eq. 4; R6).

    Omega holds the entries first in the order (|R| descending, row-major
    linear index ascending), keeping only nonzero ones.  Written as: find the
    k-th largest magnitude t; take every entry above t, then the entries
    equal to t with the smallest linear indices until k are taken.

    Returns (idx, val): idx ascending int64 linear indices, val = R.flat[idx].

    Pinned by: a brute-force full sort on tiny, tie-heavy inputs and the Eq. 4
    optimality condition (tests/test_oracle_topk.py).
    """
    a = np.abs(R).ravel()
    N = a.size
    if k <= 0 or N == 0:
        return np.zeros(0, np.int64), np.zeros(0, R.dtype)
    if k >= N:
        idx = np.flatnonzero(a > 0)
        return idx.astype(np.int64), R.ravel()[idx]
    t = np.partition(a, N - k)[N - k]           # k-th largest magnitude
    if t == 0:
        idx = np.flatnonzero(a > 0)
        return idx.astype(np.int64), R.ravel()[idx]
    above = np.flatnonzero(a > t)
    ties = np.flatnonzero(a == t)               # ascending linear index
    take = k - above.size
    idx = np.sort(np.concatenate([above, ties[:take]]))
    return idx.astype(np.int64), R.ravel()[idx]


def dense_from_support(shape, idx, val) -> np.ndarray:
    S = np.zeros(shape, dtype=np.float64)
    S.flat[idx] = val
    return S


# ---------------------------------------------------------------------------
# The GoDec loops.
# ---------------------------------------------------------------------------

@dataclass
class GoDecTrace:
    L: np.ndarray
    S: np.ndarray
    left: np.ndarray
    right: np.ndarray
    r_eff: int
    rel_err_sq: list = field(default_factory=list)     # per iteration (R7)
    e1: list = field(default_factory=list)             # ||X-L_t-S_{t-1}||^2
    e2: list = field(default_factory=list)             # ||X-L_t-S_t||^2
    supports: list = field(default_factory=list)       # idx arrays, if kept
    thresholds: list = field(default_factory=list)     # |R| of the k-th kept
    seconds: list = field(default_factory=list)        # wall time of each iteration


def godec_brp(X: np.ndarray, r: int, k: int, q: int, A1: np.ndarray,
              iters: int, eps: float | None = None,
              rank_tol: float | None = None,
              keep_supports: bool = False, lstep: str = "root",
              warm: bool = False) -> GoDecTrace:
    """Algorithm 1 (GoDec by BRP), FP64, readings R1-R7.

    lstep = "proj" takes the projection form of the L step (brp_projection)
    instead of the root form of Algorithm 1.  warm = True starts every power
    chain after the first from the previous iteration's right factor (whose
    span is that of Q2) instead of A1: a variant outside the paper (Q2 of
    the last step in the role of A1 of Sec. 3.1.1), pinned by its fixed
    point.  A1 may be a function of the iteration index t (from 0) that
    returns that iteration's draw (reading R15).

    Pinned by: on the 500 x 500 workload its trajectory equals that of the
    naive SVD GoDec (Eq. 4); the S-step half of Theorem 1 (monotone
    objective); nnz(S) = min(k, #nonzero residuals) and rank(L) <= r
    (tests/test_oracle_loop.py).
    """
    X = np.asarray(X, dtype=np.float64)
    m, n = X.shape
    S = np.zeros_like(X)
    xx = float(np.sum(X * X))
    redraw = callable(A1)
    A = np.asarray(A1(0) if redraw else A1, dtype=np.float64)[:, :r]
    tr = GoDecTrace(L=X.copy(), S=S, left=None, right=None, r_eff=r)
    for t in range(iters):
        t0 = time.perf_counter()
        if redraw and t > 0:
            A = np.asarray(A1(t), dtype=np.float64)[:, :A.shape[1]]
        D = X - S
        res = brp_projection(D, A, q) if lstep == "proj" else brp_power(D, A, q, rank_tol)
        A = res.right if warm else A[:, :res.r_eff]
        L = res.L
        tr.e1.append(float(np.sum((X - L - S) ** 2)))
        R = X - L
        idx, val = hard_threshold(R, k)
        S = dense_from_support(X.shape, idx, val)
        E = R - S
        e2 = float(np.sum(E * E))
        tr.e2.append(e2)
        tr.rel_err_sq.append(e2 / xx)
        tr.thresholds.append(float(np.min(np.abs(val))) if val.size else 0.0)
        if keep_supports:
            tr.supports.append(idx)
        tr.L, tr.S, tr.left, tr.right, tr.r_eff = L, S, res.left, res.right, res.r_eff
        tr.seconds.append(time.perf_counter() - t0)
        if eps is not None and e2 / xx <= eps:
            break
    return tr


def truncated_svd(D: np.ndarray, r: int) -> np.ndarray:
    """Best rank-r approximation: singular value hard thresholding (Eq. 4)."""
    U, s, Vt = np.linalg.svd(D, full_matrices=False)
    return (U[:, :r] * s[:r]) @ Vt[:r]


def godec_naive(X: np.ndarray, r: int, k: int, iters: int,
                keep_supports: bool = False) -> GoDecTrace:
    """Naive GoDec (Eq. 3-4): L from the truncated SVD of X - S.

    Pinned by: LAPACK's SVD is the definition of the L step; exact recovery
    of a noiseless low-rank + sparse matrix (tests/test_oracle_loop.py).
    """
    X = np.asarray(X, dtype=np.float64)
    S = np.zeros_like(X)
    xx = float(np.sum(X * X))
    tr = GoDecTrace(L=X.copy(), S=S, left=None, right=None, r_eff=r)
    for _ in range(iters):
        L = truncated_svd(X - S, r)
        tr.e1.append(float(np.sum((X - L - S) ** 2)))
        R = X - L
        idx, val = hard_threshold(R, k)
        S = dense_from_support(X.shape, idx, val)
        e2 = float(np.sum((R - S) ** 2))
        tr.e2.append(e2)
        tr.rel_err_sq.append(e2 / xx)
        if keep_supports:
            tr.supports.append(idx)
        tr.L, tr.S = L, S
    return tr


# ---------------------------------------------------------------------------
# Comparison helpers used by the parity tests.
# ---------------------------------------------------------------------------

def rel_fro(A: np.ndarray, B: np.ndarray) -> float:
    """||A - B||_F / ||B||_F (non-squared)."""
    nb = np.linalg.norm(B)
    return float(np.linalg.norm(A - B) / (nb if nb > 0 else 1.0))


def rel_fro_factors(a_left, a_right, b_left, b_right) -> float:
    """||A_l A_r^T - B_l B_r^T||_F / ||B_l B_r^T||_F without forming m x n.

    Uses ||P Q^T||_F^2 = tr((P^T P)(Q^T Q)); resolution about 1e-8 relative.
    """
    def inner(P1, Q1, P2, Q2):
        return float(np.sum((P1.T @ P2) * (Q1.T @ Q2)))
    aa = inner(a_left, a_right, a_left, a_right)
    bb = inner(b_left, b_right, b_left, b_right)
    ab = inner(a_left, a_right, b_left, b_right)
    d2 = max(aa - 2.0 * ab + bb, 0.0)
    return float(np.sqrt(d2 / bb)) if bb > 0 else float(np.sqrt(d2))
