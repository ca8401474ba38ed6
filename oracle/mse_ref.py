"""FP64 oracle of MSE training, the randomized multi-label decomposition of
Sec. 4.2.1 (test infrastructure; the GPU library never imports it).

Zhou & Tao, arXiv 1309.0302, Sec. 4.2.1 (Multi-label Subspace Ensemble,
training) and its Algorithm 4 ("MSE Training").  The training matrix X is
n x p (n samples, p features); label i is carried by the samples in the row
set Omega_i.  The model (the constrained problem of Sec. 4.2.1) is

    X = sum_i L^i + S + noise,  rank(L^i_{Omega_i}) <= r^i,
    L^i is zero outside the rows Omega_i,  card(S) <= K,

solved by alternating over the k + 1 sub-problems: for each label in turn
the rows Omega_i of X - sum_{j != i} L^j - S are replaced by a rank-r^i
approximation (bilateral random projection with A2 = Y1 and no power
scheme), then S keeps the K entries of X - sum_j L^j of largest magnitude.

Readings of the paper used here (the GPU library follows the same):

M1  Loop test.  Algorithm 4 tests ||X - sum L - S||_F^2 > eps before each
    sweep; with the initialisation below that quantity is zero on the
    labelled rows, so the loop would often not start.  As for Algorithm 1,
    the test is evaluated after each iteration, and the workloads fix the
    iteration count T.  The error reported is the squared ratio
    ||X - sum L - S||_F^2 / ||X||_F^2 (the measure of Sec. 5).
M2  A1.  Algorithm 4 draws a new standard Gaussian A1 (p x r^i) for every
    label in every iteration.  The draw for iteration t (0-based, counted
    from the start of training) and label i (0-based) is the seeded draw of
    rng_ref with seed + t * k + i (k = number of labels), modulo 2^64.
M3  Sparse step.  The printed line S := P_Phi(N) with N := |X - sum L|
    would keep magnitudes only; the sub-problem it solves (and the solution
    the section states) is S = P_Phi(X - sum_j L^j) with Phi the K entries of
    largest magnitude.  S therefore keeps the signed residual.  Phi follows
    reading R6 of godec_ref: nonzero entries only, ties broken by row-major
    linear index (smallest first).
M4  Initialisation.  Z = D^{-1} X with D = diag(Y 1), the number of labels
    of each sample; L^i_{Omega_i} := Z_{Omega_i} and S := 0.  A sample with
    no label has D_jj = 0; its row of Z is never used (it belongs to no
    Omega_i) and is taken as 0.
M5  Label update.  With N the rows Omega_i of X - sum_{j != i} L^j - S,
    Algorithm 4 sets Y1 = N A1, A2 = Y1, Y2 = N^T Y1, Y1 = N Y2 and
    L^i_{Omega_i} = Y1 (A2^T Y1)^{-1} Y2^T.  Since Y2 = N^T N A1,
    A2^T Y1 = Y2^T Y2 and L^i_{Omega_i} = N Y2 (Y2^T Y2)^{-1} Y2^T = N P_Y2,
    the projection of N's rows onto range(Y2); ``label_update`` evaluates
    this form (an orthonormal basis of range(Y2) from its SVD).  When Y2
    has numerical rank below r^i (fewer rows than r^i, or N of lower rank)
    the inverse does not exist and the projector onto range(Y2) is used
    (columns with singular value <= max(|Omega_i|, p) * 2^-52 * s_1 are
    dropped).  ``label_update_literal`` keeps the printed lines.
M6  Label order.  Within a sweep the labels are updated in index order, and
    label i sees the values the labels before it have just received
    (the for loop of Algorithm 4 as written).
M7  Output.  C^i is an orthonormal basis of the row space of L^i_{Omega_i}
    (the QR step of Algorithm 4); it is unique up to an r^i x r^i rotation,
    so results are compared through the projector C^iT C^i.

Pinned by (tests/test_oracle_mse.py): the initialisation invariant
sum_i L^i = X on labelled rows; label_update against the literal lines and
against the truncated SVD when rank(N) <= r^i, and the Theorem 3 bound of
App. II on every draw; exact recovery of a planted model with disjoint
labels in one sweep; brute-force top-K and the signed S step; the
S-step monotonicity; the label order (a replay of the last label of a sweep
against the others' final values); and with one label holding every sample
and a fixed A1 the trajectory of godec_ref.godec_brp at q = 0.
"""

import time
from dataclasses import dataclass, field

import numpy as np

from oracle.godec_ref import dense_from_support, hard_threshold
from oracle.rng_ref import a1_gaussian

_MASK = (1 << 64) - 1


def mse_a1(seed: int, t: int, i: int, k: int, p: int, r: int) -> np.ndarray:
    """A1 of iteration t and label i (reading M2): p x r standard Gaussian."""
    return a1_gaussian((seed + t * k + i) & _MASK, p, r)


def orth_range(Y: np.ndarray) -> np.ndarray:
    """Orthonormal basis of range(Y) (reading M5): left singular vectors
    whose singular value exceeds max(shape) * 2^-52 * s_1."""
    if Y.size == 0:
        return np.zeros((Y.shape[0], 0))
    U, s, _ = np.linalg.svd(Y, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return np.zeros((Y.shape[0], 0))
    keep = s > max(Y.shape) * np.finfo(np.float64).eps * s[0]
    return U[:, keep]


def label_update(N: np.ndarray, A1: np.ndarray):
    """One label's rank-r update of Algorithm 4 in its restated form
    (reading M5): L = N Q Q^T with Q an orthonormal basis of
    range(Y2), Y2 = N^T (N A1).  Returns (L, U = N Q, Q)."""
    Y1 = N @ A1
    Y2 = N.T @ Y1
    Q = orth_range(Y2)
    U = N @ Q
    return U @ Q.T, U, Q


def label_update_literal(N: np.ndarray, A1: np.ndarray) -> np.ndarray:
    """The printed lines of Algorithm 4's label update:
    Y1 = N A1, A2 = Y1, Y2 = N^T Y1, Y1 = N Y2, L = Y1 (A2^T Y1)^{-1} Y2^T."""
    Y1 = N @ A1
    A2 = Y1
    Y2 = N.T @ Y1
    Y1 = N @ Y2
    return Y1 @ np.linalg.solve(A2.T @ Y1, Y2.T)


def mse_init(X: np.ndarray, labels: list) -> list:
    """Eq. for the initialisation (reading M4): L^i_{Omega_i} = Z_{Omega_i},
    Z = D^{-1} X, D = diag(number of labels of each sample)."""
    n = X.shape[0]
    cnt = np.zeros(n)
    for rows in labels:
        cnt[rows] += 1.0
    Z = np.zeros_like(X)
    lab = cnt > 0
    Z[lab] = X[lab] / cnt[lab, None]
    return [Z[rows].copy() for rows in labels]


@dataclass
class MseTrace:
    Ls: list                                           # L^i_{Omega_i}, n_i x p
    U: list                                            # N Q of the last update
    Q: list                                            # p x r_i' bases (C^i)^T
    S: np.ndarray                                      # dense n x p
    R: np.ndarray | None = None                        # X - sum L of the last S step
    rel_err_sq: list = field(default_factory=list)     # per iteration (M1)
    thresholds: list = field(default_factory=list)     # |R| of the K-th kept
    supports: list = field(default_factory=list)       # idx arrays, if kept
    seconds: list = field(default_factory=list)        # wall time per iteration


def embed_sum(n: int, p: int, labels: list, Ls: list) -> np.ndarray:
    """sum_i L^i as a dense n x p matrix (each L^i zero off Omega_i),
    accumulated in label order."""
    T = np.zeros((n, p))
    for rows, L in zip(labels, Ls):
        T[rows] += L
    return T


def mse_train(X: np.ndarray, labels: list, ranks: list, K: int, seed: int,
              iters: int, state=None, t0: int = 0, keep_supports: bool = False,
              a1_fn=None) -> MseTrace:
    """Algorithm 4 (MSE training), FP64, readings M1-M7.

    labels: list of k ascending int arrays (the row sets Omega_i); ranks:
    the bounds r^i; K: the cardinality bound of S.  state = (Ls, S) starts
    from a given state instead of the initialisation (per-step checks), with
    t0 the index of its first iteration (for the A1 draws).  a1_fn(t, i, p,
    r) overrides the seeded draw of reading M2.
    """
    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    k = len(labels)
    if a1_fn is None:
        def a1_fn(t, i, pp, rr):
            return mse_a1(seed, t, i, k, pp, rr)
    if state is None:
        Ls = mse_init(X, labels)
        S = np.zeros_like(X)
    else:
        Ls = [np.asarray(L, dtype=np.float64).copy() for L in state[0]]
        S = np.asarray(state[1], dtype=np.float64).copy()
    xx = float(np.sum(X * X))
    tr = MseTrace(Ls=Ls, U=[None] * k, Q=[None] * k, S=S)
    T = embed_sum(n, p, labels, Ls)                # sum_j L^j, kept up to date
    for t in range(t0, t0 + iters):
        tic = time.perf_counter()
        for i in range(k):
            rows = labels[i]
            # N := (X - sum_{j != i} L^j - S)_{Omega_i}, with the labels
            # before i already updated in this sweep (reading M6)
            N = (X - T - S)[rows] + Ls[i]
            L, U, Q = label_update(N, a1_fn(t, i, p, ranks[i]))
            T[rows] += L - Ls[i]
            Ls[i] = L
            tr.U[i], tr.Q[i] = U, Q
        R = X - T                                  # X - sum_j L^j
        idx, val = hard_threshold(R, K)            # signed (reading M3)
        S = dense_from_support(X.shape, idx, val)
        E = R - S
        tr.rel_err_sq.append(float(np.sum(E * E)) / xx)
        tr.thresholds.append(float(np.min(np.abs(val))) if val.size else 0.0)
        if keep_supports:
            tr.supports.append(idx)
        tr.S, tr.R = S, R
        tr.seconds.append(time.perf_counter() - tic)
    tr.Ls = Ls
    return tr


def basis(L: np.ndarray) -> np.ndarray:
    """C^i of Algorithm 4's output step: QR of (L^i_{Omega_i})^T, keeping the
    columns of Q that span its range (reading M7); returned as p x r'."""
    return orth_range(L.T)
