"""FP64 oracle of GoDec matrix completion (test infrastructure).

Sec. 2 of Zhou & Tao (arXiv 1309.0302) notes that GoDec yields a matrix
completion algorithm by replacing the cardinality constraint of the S update
with a fixed support set.  This module is that variant of Algorithm 1, with
the same power-scheme L update (``godec_ref.brp_power``).  Only the tests
use it; the GPU library never does.

Readings:

C1  The fixed support Omega_bar is the set of unobserved entries.  The S
    update is S_t = P_Omega_bar(X - L_t): S takes the whole residual there, so
    D = X - S_t equals X on the observed entries and L_t on the unobserved
    ones (the imputation).  The values X holds at unobserved entries do not
    affect L after the first iteration.
C2  The relative error is ||X - L - S||_F^2 / ||X||_F^2 (Sec. 5), which is the
    squared error on the observed entries over ||X||_F^2.
C3  The support is given as ascending row-major linear indices i*n + j.

Pinning status (tests/test_oracle_completion.py): pinned (exact recovery of
a rank-r matrix from 70 % of its entries; the D imputation invariant; the
S step zeroes the residual on the support; with an empty support every
iteration equals brp_power on X; planted mistakes are caught).
"""

from dataclasses import dataclass, field

import numpy as np

from . import godec_ref


@dataclass
class CompletionTrace:
    L: np.ndarray
    S: np.ndarray
    left: np.ndarray
    right: np.ndarray
    r_eff: int
    rel_err_sq: list = field(default_factory=list)


def fixed_support_step(R: np.ndarray, support: np.ndarray) -> np.ndarray:
    """S = P_Omega_bar(R): R on the support, zero elsewhere (reading C1)."""
    S = np.zeros_like(R)
    S.flat[support] = R.flat[support]
    return S


def godec_completion(X, r, q, A1, support, iters, eps=None, rank_tol=None):
    """Algorithm 1 with the S update on a fixed support (readings C1-C3).
    A1 may be a function of the iteration index t (from 0) that returns that
    iteration's draw (godec_ref's reading R15)."""
    X = np.asarray(X, dtype=np.float64)
    support = np.asarray(support, dtype=np.int64)
    S = np.zeros_like(X)
    xx = float(np.sum(X * X))
    redraw = callable(A1)
    A = np.asarray(A1(0) if redraw else A1, dtype=np.float64)[:, :r]
    tr = CompletionTrace(L=X.copy(), S=S, left=None, right=None, r_eff=r)
    for t in range(iters):
        if redraw and t > 0:
            A = np.asarray(A1(t), dtype=np.float64)[:, :A.shape[1]]
        res = godec_ref.brp_power(X - S, A, q, rank_tol)
        A = A[:, :res.r_eff]
        R = X - res.L
        S = fixed_support_step(R, support)
        E = R - S
        tr.rel_err_sq.append(float(np.sum(E * E)) / xx)
        tr.L, tr.S, tr.left, tr.right, tr.r_eff = res.L, S, res.left, res.right, res.r_eff
        if eps is not None and tr.rel_err_sq[-1] <= eps:
            break
    return tr
