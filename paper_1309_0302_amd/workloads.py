"""Seeded synthetic inputs for GoDec (shared by the tests, the benchmark and
the oracle checks).  This module holds no step of the decomposition itself:
it only builds X = L0 + S0 + G matrices and the problem parameters.

The recipes follow the synthetic setup of Sec. 5.1 of the paper (low-rank part
as a product of two Gaussian factors, sparse part on a uniformly drawn entry
set, dense Gaussian noise) at the sizes of the five workloads below.  In the
``N(0, v)`` notation of the workload descriptions the second argument is the
variance; the standard deviation actually used is recorded in each returned
``Workload.recipe``.

W1  500 x 500 FP64: U, V 500 x 5 iid N(0,1); 5% support (12 500 entries) at
    uniform positions with values U[-10, 10]; noise std sqrt(1e-3);
    r = 5, k = 12 500, q = 2, T = 20.
W2  25 344 x 200 FP32, a video-shaped matrix (144 x 176 pixels x 200
    frames) standing in for the surveillance sequences of Sec. 5.2: a rank-2
    background U V^T / max(U V^T) with U, V iid U[0,1]; 8 moving 16 x 16
    blocks per frame with additive offsets U[0.3, 0.7]; noise std
    sqrt(1e-3); r = 2, k = 0.08 m n, q = 1, T = 50.
W3  10 000 x 10 000 FP32: U, V iid N(0, var 1/sqrt(20)) (unit-variance
    U V^T entries); 2% support (2e6 entries) with values U[-5, 5]; noise std
    0.01; r = 20, k = 2e6, q = 2, T = 30.
W4  64 independent FP32 problems: m ~ U{2000..20000}, n ~ U{100..400},
    r ~ U{1..8}, support fraction ~ U[0.03, 0.10] with values U[-5, 5],
    noise std sqrt(1e-3); q = 1, T = 25.
W5  16 FP32 problems of 4096 x 256, r = 4, 5% support, q = 1, T = 10,
    with Gaussian targets for a loss on (L, S).

GreBsmo (Sec. 3.2.1) workloads, with the parameters a GreBsmo run takes
(rank bound r, rows per stage dr, inner iterations K, soft threshold lam,
power steps) in ``GreBsmoWorkload``:
G1  500 x 500 FP64 planted problem (the shape of the phase-diagram
    experiment of Sec. 5.4): U, V iid N(0, var 1/sqrt(r)) with r = 5,
    5% support of values +-5 (random signs), no noise; r = 5, dr = 1,
    K = 30, lam = 0.1, power = 2.
Matrix completion (Sec. 2, fixed support) workload:
M1  the W3 matrix (10 000 x 10 000 FP32, r = 20, q = 2) with a seeded 10 %
    of its entries unobserved (``missing_support``).

MSE1, MSE2  multi-label training matrices for MSE training (Sec. 4.2.1),
    standing in for the multi-label datasets of Sec. 5 (not available):
    n samples x p features; each of k labels is carried by each sample with
    probability `label_prob` (a sample with none gets one label drawn
    uniformly); label i has rank r_i ~ U{2 .. rmax} and contributes
    U_i V_i^T on its rows with U_i, V_i iid N(0, var 1/sqrt(r_i)) (unit
    variance entries); 2% sparse entries U[-5, 5]; noise std 1e-3;
    K = the sparse support size.
    MSE1: n = 2048, p = 128, k = 8, rmax = 6, label_prob 0.2, T = 10.
    MSE2: n = 65 536, p = 512, k = 32, rmax = 8, label_prob 0.1, T = 10.

G2  25 344 x 500 FP32 video-shaped matrix (144 x 176 pixels x 500 frames,
    the shape of the Hall sequence of Sec. 5.5) from the W2 recipe with 500
    frames; r = 4, dr = 1, K = 10, lam = 0.125, power = 2.
"""

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    X: np.ndarray
    r: int
    k: int
    q: int
    iters: int
    seed: int
    recipe: dict = field(default_factory=dict)
    L0: np.ndarray | None = None
    S0_idx: np.ndarray | None = None


def round_half_up(x: float) -> int:
    return int(np.floor(x + 0.5))


def lowrank_sparse(m: int, n: int, r: int, *, factor_std: float,
                   support: int, amp: float, noise_std: float,
                   seed: int, dtype=np.float64, keep_parts: bool = False):
    """X = U V^T + P_Omega(values) + noise, built in FP64 then cast once."""
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((m, r)) * factor_std
    V = rng.standard_normal((n, r)) * factor_std
    X = U @ V.T
    L0 = X.copy() if keep_parts else None
    idx = rng.choice(m * n, size=support, replace=False) if support > 0 \
        else np.zeros(0, np.int64)
    vals = rng.uniform(-amp, amp, size=support)
    X.flat[idx] += vals
    if noise_std > 0:
        X += rng.standard_normal((m, n)) * noise_std
    return X.astype(dtype, copy=False), L0, np.sort(idx)


def w1(seed: int = 1001) -> Workload:
    m = n = 500
    X, L0, sidx = lowrank_sparse(m, n, 5, factor_std=1.0, support=12500,
                                 amp=10.0, noise_std=np.sqrt(1e-3), seed=seed,
                                 keep_parts=True)
    return Workload("w1_500x500_f64", X, 5, 12500, 2, 20, seed,
                    dict(factor_std=1.0, support=12500, amp=10.0,
                         noise_std=float(np.sqrt(1e-3)), dtype="f64"),
                    L0, sidx)


def video_background_blocks(seed: int = 1002, height: int = 144,
                            width: int = 176, frames: int = 200,
                            blocks: int = 8, block: int = 16,
                            noise_std: float = float(np.sqrt(1e-3))):
    """Video-shaped matrix: pixels (row y*width + x) by frames."""
    rng = np.random.default_rng(seed)
    m = height * width
    U = rng.uniform(0.0, 1.0, size=(m, 2))
    V = rng.uniform(0.0, 1.0, size=(frames, 2))
    B = U @ V.T
    B /= B.max()
    X = B.copy()
    mask = np.zeros((m, frames), dtype=bool)
    pos = np.stack([rng.integers(0, height - block + 1, blocks),
                    rng.integers(0, width - block + 1, blocks)], axis=1)
    vel = np.zeros((blocks, 2), dtype=np.int64)
    for b in range(blocks):
        while True:
            v = rng.integers(-3, 4, size=2)
            if v[0] != 0 or v[1] != 0:
                vel[b] = v
                break
    offs = rng.uniform(0.3, 0.7, size=blocks)
    lim = np.array([height - block, width - block])
    for f in range(frames):
        frame = np.zeros((height, width), dtype=bool)
        add = np.zeros((height, width))
        for b in range(blocks):
            y, x = pos[b]
            frame[y:y + block, x:x + block] = True
            add[y:y + block, x:x + block] += offs[b]
        mask[:, f] = frame.ravel()
        X[:, f] += add.ravel()
        # move with reflection at the borders
        for d in range(2):
            nxt = pos[:, d] + vel[:, d]
            over = (nxt < 0) | (nxt > lim[d])
            vel[over, d] = -vel[over, d]
            pos[:, d] = pos[:, d] + vel[:, d]
    X += rng.standard_normal((m, frames)) * noise_std
    return X, B, mask


def w2(seed: int = 1002) -> Workload:
    X, B, mask = video_background_blocks(seed)
    m, n = X.shape
    k = round_half_up(0.08 * m * n)
    return Workload("w2_video_25344x200_f32", X.astype(np.float32), 2, k, 1,
                    50, seed,
                    dict(background="UV^T/max, U,V ~ U[0,1]", blocks=8,
                         block=16, offsets="U[0.3,0.7]",
                         noise_std=float(np.sqrt(1e-3)),
                         support_fraction=float(mask.mean()), dtype="f32"),
                    B, np.flatnonzero(mask.ravel()))


def w3(seed: int = 1003, m: int = 10000, n: int = 10000, r: int = 20,
       support: int | None = None, dtype=np.float32) -> Workload:
    if support is None:
        support = round_half_up(0.02 * m * n)
    std = (1.0 / np.sqrt(r)) ** 0.5
    X, _, sidx = lowrank_sparse(m, n, r, factor_std=std, support=support,
                                amp=5.0, noise_std=0.01, seed=seed,
                                dtype=dtype)
    return Workload(f"w3_{m}x{n}_r{r}", X, r, support, 2, 30, seed,
                    dict(factor_std=float(std), support=support, amp=5.0,
                         noise_std=0.01, dtype=np.dtype(dtype).name),
                    None, sidx)


def w4(seed: int = 1004, count: int = 64) -> list[Workload]:
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        m = int(rng.integers(2000, 20001))
        n = int(rng.integers(100, 401))
        r = int(rng.integers(1, 9))
        rho = float(rng.uniform(0.03, 0.10))
        k = round_half_up(rho * m * n)
        sub = int(rng.integers(0, 2 ** 31))
        std = (1.0 / np.sqrt(r)) ** 0.5
        X, _, sidx = lowrank_sparse(m, n, r, factor_std=std, support=k,
                                    amp=5.0, noise_std=float(np.sqrt(1e-3)),
                                    seed=sub, dtype=np.float32)
        out.append(Workload(f"w4_{i}_{m}x{n}_r{r}", X, r, k, 1, 25, sub,
                            dict(rho=rho), None, sidx))
    return out


def w5(seed: int = 1005, batch: int = 16, m: int = 4096, n: int = 256,
       r: int = 4, iters: int = 10, dtype=np.float32):
    rng = np.random.default_rng(seed)
    k = round_half_up(0.05 * m * n)
    std = (1.0 / np.sqrt(r)) ** 0.5
    Xs, Lt, St = [], [], []
    for b in range(batch):
        sub = int(rng.integers(0, 2 ** 31))
        X, _, _ = lowrank_sparse(m, n, r, factor_std=std, support=k, amp=5.0,
                                 noise_std=float(np.sqrt(1e-3)), seed=sub,
                                 dtype=dtype)
        Xs.append(X)
        Lt.append(rng.standard_normal((m, n)).astype(dtype))
        St.append(rng.standard_normal((m, n)).astype(dtype))
    return dict(X=np.stack(Xs), L_target=np.stack(Lt), S_target=np.stack(St),
                r=r, k=k, q=1, iters=iters, seed=seed)


def tiny(m: int, n: int, r: int, *, rho: float = 0.05, amp: float = 5.0,
         noise_std: float = 1e-3, seed: int = 0, dtype=np.float64,
         factor_std: float = 1.0) -> Workload:
    support = round_half_up(rho * m * n)
    X, L0, sidx = lowrank_sparse(m, n, r, factor_std=factor_std,
                                 support=support, amp=amp,
                                 noise_std=noise_std, seed=seed, dtype=dtype,
                                 keep_parts=True)
    return Workload(f"tiny_{m}x{n}_r{r}", X, r, support, 1, 5, seed, {}, L0,
                    sidx)


@dataclass
class GreBsmoWorkload:
    name: str
    X: np.ndarray
    r: int
    dr: int
    K: int
    lam: float
    power: int
    seed: int
    recipe: dict = field(default_factory=dict)
    L0: np.ndarray | None = None


def planted_pm(m: int, n: int, r: int, *, rho: float, amp: float, seed: int,
               dtype=np.float64):
    """X = U V^T + S0, S0 = +-amp on a Bernoulli(rho) support (no noise)."""
    rng = np.random.default_rng(seed)
    std = (1.0 / np.sqrt(r)) ** 0.5
    U = rng.standard_normal((m, r)) * std
    V = rng.standard_normal((n, r)) * std
    L0 = U @ V.T
    u = rng.uniform(size=(m, n))
    S0 = np.where(u < rho / 2, amp, np.where(u < rho, -amp, 0.0))
    return (L0 + S0).astype(dtype), L0, S0


def g1(seed: int = 1006) -> GreBsmoWorkload:
    X, L0, _ = planted_pm(500, 500, 5, rho=0.05, amp=5.0, seed=seed)
    return GreBsmoWorkload("g1_planted_500x500_f64", X, 5, 1, 30, 0.1, 2, seed,
                           dict(rho=0.05, amp=5.0, dtype="f64"), L0)


def g2(seed: int = 1007, frames: int = 500) -> GreBsmoWorkload:
    X, B, mask = video_background_blocks(seed, frames=frames)
    return GreBsmoWorkload(f"g2_video_25344x{frames}_f32", X.astype(np.float32), 4, 1, 10,
                           0.125, 2, seed,
                           dict(frames=frames, support_fraction=float(mask.mean()),
                                dtype="f32"), B)


def missing_support(m: int, n: int, frac: float, seed: int,
                    chunk: int = 1 << 24) -> np.ndarray:
    """Ascending linear indices of a Bernoulli(frac) set of unobserved
    entries of an m x n matrix, drawn chunk by chunk (bounded memory)."""
    rng = np.random.default_rng(seed)
    out = []
    total = m * n
    for c0 in range(0, total, chunk):
        c1 = min(c0 + chunk, total)
        out.append(np.flatnonzero(rng.random(c1 - c0) < frac).astype(np.int64) + c0)
    return np.concatenate(out) if out else np.zeros(0, np.int64)


@dataclass
class MseWorkload:
    name: str
    X: np.ndarray
    labels: list          # k ascending int64 row sets Omega_i
    ranks: list           # r_i
    K: int
    iters: int
    seed: int
    recipe: dict = field(default_factory=dict)


def multilabel(n: int, p: int, k: int, *, rmax: int, label_prob: float,
               support_frac: float = 0.02, amp: float = 5.0,
               noise_std: float = 1e-3, seed: int, dtype=np.float64,
               iters: int = 10, name: str | None = None) -> MseWorkload:
    """X = sum_i (rows Omega_i: U_i V_i^T) + sparse + noise with random label
    sets (the MSE model of Sec. 4.2.1), built in FP64 and cast once."""
    rng = np.random.default_rng(seed)
    Y = rng.random((n, k)) < label_prob
    none = np.flatnonzero(~Y.any(axis=1))
    Y[none, rng.integers(0, k, size=none.size)] = True
    ranks = [int(v) for v in rng.integers(2, rmax + 1, size=k)]
    X = np.zeros((n, p))
    labels = []
    for i in range(k):
        rows = np.flatnonzero(Y[:, i]).astype(np.int64)
        std = (1.0 / np.sqrt(ranks[i])) ** 0.5
        U = rng.standard_normal((rows.size, ranks[i])) * std
        V = rng.standard_normal((p, ranks[i])) * std
        X[rows] += U @ V.T
        labels.append(rows)
    K = round_half_up(support_frac * n * p)
    idx = rng.choice(n * p, size=K, replace=False)
    X.flat[idx] += rng.uniform(-amp, amp, size=K)
    X += rng.standard_normal((n, p)) * noise_std
    return MseWorkload(name or f"mse_{n}x{p}_k{k}", X.astype(dtype, copy=False), labels,
                       ranks, K, iters, seed,
                       dict(label_prob=label_prob, rmax=rmax, support_frac=support_frac,
                            amp=amp, noise_std=noise_std, dtype=np.dtype(dtype).name))


def mse1(seed: int = 1010, dtype=np.float64) -> MseWorkload:
    return multilabel(2048, 128, 8, rmax=6, label_prob=0.2, seed=seed, dtype=dtype,
                      name="mse1_2048x128_k8")


def mse2(seed: int = 1011, dtype=np.float32) -> MseWorkload:
    return multilabel(65536, 512, 32, rmax=8, label_prob=0.1, seed=seed, dtype=dtype,
                      name="mse2_65536x512_k32")
