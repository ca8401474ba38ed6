"""FP64 oracle of GreBsmo, greedy bilateral smoothing (test infrastructure).

Zhou & Tao, "Unmixing Incoherent Structures of Big Data by Randomized or
Greedy Decomposition", arXiv 1309.0302, Sec. 3.2 (the GreB paradigm,
Algorithm 2) and Sec. 3.2.1 (GreBsmo: the model Eq. 10, its alternating
rules Eq. 11, the soft-thresholding operator Eq. 12, the QR form Eq. 13 and
the greedy direction Eq. 14).  Plain NumPy / LAPACK in float64, written to be
read against the paper.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark use it; the GPU library never does.

Notation: X is m x n, L = U V with U m x r_i and V r_i x n, S the sparse
part, lambda the soft threshold, dr the rank step, K the inner iterations
per rank, power the number of power steps of the random-projection estimate
of the greedy directions.

Readings of the paper (where it is silent or ambiguous) used here:

G1  Algorithm 2's loop test is printed as "residual error <= tau"; it is read
    as "repeat while the relative error exceeds tau", and the rank bound r of
    Eq. 10 also ends the loop.  The test is made after each rank stage.
G2  V starts empty: the first dr rows come from the same greedy step applied
    to X - U V - S with U V = 0 and S = 0, i.e. to X itself.
G3  The added rows span the top-dr right singular subspace of
    dF/dV = X - U V - S (Eq. 14), estimated by random projections as the
    paper allows: an orthonormal basis of (R^T R)^power Omega, with R the
    derivative, Omega an n x dr standard Gaussian block and power >= 1;
    every power step is re-orthonormalised (the span is unchanged).  Stage
    s uses columns [s dr, min((s+1) dr, r)) of one n x r Gaussian matrix
    drawn from the seed.
G4  The S update is Eq. 12 with the threshold lambda as given.  Eq. 12 is
    the exact minimiser of 1/2 ||X - U V - S||_F^2 + lambda ||S||_1, so that
    is the objective F used for the monotonicity pins (with Eq. 10's
    unhalved first term the minimiser would threshold at lambda / 2).
G5  Each stage runs exactly K inner iterations of Eq. 13 (the "or until the
    object converges" alternative is not used), so the schedule is fixed.
G6  The relative error is ||X - U V - S||_F^2 / ||X||_F^2, the definition of
    Sec. 5.
G7  U = Q is any orthonormal basis of range((X - S) V^T): U V = Q Q^T (X - S)
    does not depend on which one.  The oracle uses LAPACK's Householder QR.

Pinning status (the tests under tests/test_oracle_grebsmo.py):
    soft_threshold     pinned (brute-force scalar minimisation of the Eq. 12
                       objective; hand-worked values)
    inner_step         pinned (equals the alternating least-squares rules of
                       Eq. 11 with pseudo-inverses; S-step KKT conditions;
                       F non-increasing)
    greedy_directions  pinned (LAPACK SVD's top right singular vectors on an
                       input with a spectral gap)
    grebsmo_stage,
    grebsmo            pinned (F non-increasing across stages; truncated SVD
                       when lambda is so large that S stays 0; recovery of a
                       planted low-rank + sparse X, the success criterion of
                       Sec. 5.4)
"""

from dataclasses import dataclass, field

import numpy as np


def soft_threshold(R: np.ndarray, lam: float) -> np.ndarray:
    """Element-wise soft thresholding S_lambda (Eq. 12)."""
    return np.sign(R) * np.maximum(np.abs(R) - lam, 0.0)


def objective(X, L, S, lam) -> float:
    """F = 1/2 ||X - L - S||_F^2 + lambda ||S||_1 (Eq. 10; reading G4)."""
    E = X - L - S
    return 0.5 * float(np.sum(E * E)) + lam * float(np.sum(np.abs(S)))


def orth(A: np.ndarray) -> np.ndarray:
    """Orthonormal basis of range(A) (thin Householder QR; reading G7)."""
    Q, _ = np.linalg.qr(A, mode="reduced")
    return Q


def inner_step(X, S, V, lam):
    """One pass of Eq. 13: U = Q with QR((X - S) V^T) = Q R, V = Q^T (X - S),
    S = S_lambda(X - U V).  Returns (U, V, S)."""
    D = X - S
    U = orth(D @ V.T)
    V = U.T @ D
    S = soft_threshold(X - U @ V, lam)
    return U, V, S


def inner_step_als(X, S, V, lam):
    """Eq. 11, the alternating least-squares rules with pseudo-inverses (the
    form Eq. 13 replaces; used only to pin ``inner_step``)."""
    D = X - S
    U = D @ V.T @ np.linalg.pinv(V @ V.T)
    V = np.linalg.pinv(U.T @ U) @ U.T @ D
    S = soft_threshold(X - U @ V, lam)
    return U, V, S


def greedy_directions(R: np.ndarray, Omega: np.ndarray, power: int) -> np.ndarray:
    """Rows to append to V: an orthonormal basis (as rows) of
    (R^T R)^power Omega, the random-projection estimate of the top right
    singular vectors of R = dF/dV (Eq. 14; reading G3)."""
    if power < 1:
        raise ValueError("power must be >= 1")
    Z = Omega
    for _ in range(power):
        Z = orth(R.T @ (R @ Z))
    return Z.T


@dataclass
class GreBsmoResult:
    U: np.ndarray
    V: np.ndarray
    S: np.ndarray
    rel_err: list = field(default_factory=list)     # after each stage (G6)
    ranks: list = field(default_factory=list)       # rank after each stage
    objective: list = field(default_factory=list)   # F after every inner step
    added: list = field(default_factory=list)       # rows appended by each stage
    states: list = field(default_factory=list)      # (U, V, S) after each stage


def stage_columns(stage: int, dr: int, r: int) -> tuple[int, int]:
    """Columns of the seed's Gaussian matrix that stage ``stage`` uses (G3)."""
    c0 = stage * dr
    return c0, min(c0 + dr, r)


def grebsmo_stage(X, U, V, S, Omega_s, K, lam, power, objective_log=None):
    """One rank stage of Algorithm 2 from the state (U, V, S): append the
    greedy rows for dF/dV = X - U V - S (Eq. 14; readings G2, G3), then K
    inner iterations of Eq. 13 (G5).  Returns (U, V, S, Z) with Z the rows
    appended."""
    R = X - U @ V - S
    Z = greedy_directions(R, Omega_s, power)
    V = np.vstack([V, Z])
    for _ in range(K):
        U, V, S = inner_step(X, S, V, lam)
        if objective_log is not None:
            objective_log.append(objective(X, U @ V, S, lam))
    return U, V, S, Z


def grebsmo(X: np.ndarray, r: int, dr: int, K: int, lam: float, power: int,
            Omega: np.ndarray, tau: float = 0.0, stages: int | None = None,
            track: bool = False) -> GreBsmoResult:
    """GreBsmo (Algorithm 2 with the Eq. 13 updates), readings G1-G7.

    Omega is the n x r Gaussian matrix of reading G3.  ``stages`` caps the
    number of rank stages (None: until the rank reaches r or the relative
    error reaches tau).  With ``track`` the objective F is recorded after
    every inner iteration, and the rows each stage appended and the state
    (U, V, S) at the end of each stage are kept.
    """
    m, n = X.shape
    if Omega.shape != (n, r):
        raise ValueError("Omega must be n x r")
    S = np.zeros_like(X)
    U = np.zeros((m, 0))
    V = np.zeros((0, n))
    normx2 = float(np.sum(X * X))
    res = GreBsmoResult(U, V, S)
    stage = 0
    while True:
        c0, c1 = stage_columns(stage, dr, r)
        U, V, S, Z = grebsmo_stage(X, U, V, S, Omega[:, c0:c1], K, lam, power,
                                   res.objective if track else None)
        E = X - U @ V - S
        res.rel_err.append(float(np.sum(E * E)) / normx2)
        res.ranks.append(V.shape[0])
        if track:
            res.added.append(Z)
            res.states.append((U, V, S))
        stage += 1
        if V.shape[0] >= r or res.rel_err[-1] <= tau:
            break
        if stages is not None and stage >= stages:
            break
    res.U, res.V, res.S = U, V, S
    return res
