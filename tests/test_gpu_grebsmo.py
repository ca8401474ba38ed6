"""GPU parity of GreBsmo (Sec. 3.2.1) against the FP64 oracle, through the
C ABI.

FP64: the whole trajectory (every stage's relative error, the final L = U V
and S) must match the oracle run on the same X and the same Omega within
1e-12 (relative Frobenius for L, max-abs relative to max |X| for S; measured
at most 2.1e-15).  The soft threshold is continuous, so no discrete decision
can make the two runs part ways; only rounding differs.

FP32: per-stage parity from the GPU's own state.  After every GPU stage the
oracle runs the same stage in FP64 from the state (U, V, S) the GPU held
before it, with the same Omega block, and the GPU's new L and S must match
within 1e-5 (relative Frobenius for L; max-abs relative to max |X| for S;
measured at most 3.9e-7).  The bound: each panel product accumulates FP32
roundings over at most 25 344 terms (at worst sqrt(m) 2^-24 ~ 1e-5, at the
observed random-walk rate far less), the bases come from an FP64 Gram
matrix, and the K steps of a stage are contractive on the error of the step
before.
"""
import numpy as np
import pytest

from oracle import grebsmo_ref as g
from oracle import rng_ref
from paper_1309_0302_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(X):
    return torch.from_numpy(np.ascontiguousarray(X)).cuda()


def state(gb):
    U, Vt = gb.factors()
    S = gb.S()
    torch.cuda.synchronize()
    return (U.cpu().numpy().astype(np.float64), Vt.cpu().numpy().astype(np.float64).T,
            S.cpu().numpy().astype(np.float64))


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def problem(m, n, r, seed, rho=0.05, amp=5.0, noise=1e-2, dtype=np.float64):
    X, L0, _ = wl.planted_pm(m, n, r, rho=rho, amp=amp, seed=seed)
    X = X + noise * np.random.default_rng(seed + 1).standard_normal((m, n))
    return X.astype(dtype), L0


def run_f64(X, r, dr, K, lam, power, seed, tol=1e-12):
    from paper_1309_0302_amd.binding import GreBsmo
    print(f"\n[grebsmo f64] shape={X.shape} r={r} dr={dr} K={K} lam={lam} power={power}",
          flush=True)
    Om = rng_ref.a1_gaussian(seed, X.shape[1], r)
    ref = g.grebsmo(X, r, dr, K, lam, power, Om)
    gb = GreBsmo(dev(X), r, dr=dr, power=power, lam=lam, seed=seed)
    errs = []
    for s in range(len(ref.rel_err)):
        gb.stage(K)
        info = gb.info()
        assert info.rank == ref.ranks[s]
        errs.append(abs(info.rel_err_sq - ref.rel_err[s]) / max(ref.rel_err[s], 1e-300))
    U, V, S = state(gb)
    eL = rel(U @ V, ref.U @ ref.V)
    eS = np.max(np.abs(S - ref.S)) / np.max(np.abs(X))
    nnz_ref = int(np.count_nonzero(ref.S))
    print(f"  rel_err parity {max(errs):.2e}  L {eL:.2e}  S {eS:.2e}  nnz {info.nnz}/{nnz_ref}",
          flush=True)
    assert max(errs) <= tol and eL <= tol and eS <= tol
    assert abs(info.nnz - nnz_ref) <= max(2, nnz_ref // 10000)
    gb.close()
    return ref


@pytest.mark.parametrize("m,n,r,dr,K,lam", [
    (300, 200, 6, 2, 4, 0.1),
    (333, 257, 5, 1, 3, 0.25),      # ragged rows and a ragged column tile
    (150, 400, 4, 3, 3, 0.1),       # m < n; last stage appends 1 row
    (20, 10, 2, 1, 2, 0.05),        # tiny
])
def test_f64_trajectory_matches_oracle(m, n, r, dr, K, lam):
    X, _ = problem(m, n, r, seed=m + n)
    run_f64(X, r, dr, K, lam, 2, seed=m * 7 + n)


def test_f64_single_stage_when_dr_exceeds_r():
    X, _ = problem(120, 90, 3, seed=5)
    ref = run_f64(X, 3, 5, 4, 0.2, 2, seed=6)
    assert ref.ranks == [3]


def test_f64_huge_lambda_keeps_s_zero():
    X, _ = problem(200, 120, 3, seed=8)
    ref = run_f64(X, 3, 1, 6, 1e30, 2, seed=9)
    assert not ref.S.any()


def test_f64_lambda_zero_single_stage():
    """lambda = 0: S = X - U V, so the residual vanishes."""
    from paper_1309_0302_amd.binding import GreBsmo
    X, _ = problem(100, 80, 2, seed=10)
    gb = GreBsmo(dev(X), 2, dr=2, power=2, lam=0.0, seed=11)
    gb.stage(3)
    info = gb.info()
    assert info.rel_err_sq == 0.0
    U, V, S = state(gb)
    assert np.max(np.abs(S + U @ V - X)) <= 1e-12 * np.max(np.abs(X))
    gb.close()


def per_stage_f32(X, r, dr, K, lam, power, seed, tol=1e-5):
    from paper_1309_0302_amd.binding import GreBsmo
    print(f"\n[grebsmo f32] shape={X.shape} r={r} dr={dr} K={K} lam={lam}", flush=True)
    n = X.shape[1]
    Om = rng_ref.a1_gaussian(seed, n, r)
    X64 = X.astype(np.float64)
    gb = GreBsmo(dev(X), r, dr=dr, power=power, lam=lam, seed=seed)
    U = np.zeros((X.shape[0], 0))
    V = np.zeros((0, n))
    S = np.zeros_like(X64)
    worst = (0.0, 0.0)
    stage = 0
    while True:
        c0, c1 = g.stage_columns(stage, dr, r)
        Uo, Vo, So, _ = g.grebsmo_stage(X64, U, V, S, Om[:, c0:c1], K, lam, power)
        gb.stage(K)
        U, V, S = state(gb)
        eL = rel(U @ V, Uo @ Vo)
        eS = np.max(np.abs(S - So)) / np.max(np.abs(X64))
        print(f"  stage {stage}: L {eL:.2e}  S {eS:.2e}", flush=True)
        worst = (max(worst[0], eL), max(worst[1], eS))
        stage += 1
        if c1 >= r:
            break
    assert worst[0] <= tol and worst[1] <= tol, worst
    info = gb.info()
    E = X64 - U @ V - S
    assert abs(info.rel_err_sq - np.sum(E * E) / np.sum(X64 * X64)) <= 1e-3 * info.rel_err_sq
    assert info.nnz == np.count_nonzero(S)
    gb.close()


@pytest.mark.parametrize("m,n,r,dr,K,lam", [
    (300, 200, 6, 2, 4, 0.1),
    (333, 257, 5, 1, 3, 0.25),
    (150, 400, 4, 3, 3, 0.1),
    (1000, 300, 8, 2, 5, 0.125),
    (700, 400, 12, 4, 3, 0.1),      # r > 8: the unfused soft pass + D V^T pass
    (500, 260, 1, 1, 4, 0.1),       # one-column panels
    (500, 260, 2, 2, 3, 0.1),
    (20, 10, 2, 1, 3, 0.05),        # smaller than one tile in both directions
])
def test_f32_per_stage_parity(m, n, r, dr, K, lam):
    X, _ = problem(m, n, r, seed=m + n, dtype=np.float32)
    per_stage_f32(X, r, dr, K, lam, 2, seed=m * 7 + n)


def test_f32_video_full_size_per_stage_parity():
    """The 25 344 x 500 video-shaped workload, in the launch configuration
    the benchmark times."""
    w = wl.g2()
    per_stage_f32(w.X, w.r, w.dr, w.K, w.lam, w.power, seed=w.seed)


def test_results_are_bitwise_reproducible():
    from paper_1309_0302_amd.binding import GreBsmo
    X, _ = problem(500, 300, 4, seed=12, dtype=np.float32)
    outs = []
    for _ in range(2):
        gb = GreBsmo(dev(X), 4, dr=1, power=2, lam=0.1, seed=13)
        gb.solve(4)
        outs.append(state(gb))
        gb.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_tau_stops_like_the_oracle():
    from paper_1309_0302_amd.binding import GreBsmo
    X, _ = problem(240, 160, 2, seed=14)
    Om = rng_ref.a1_gaussian(15, 160, 6)
    full = g.grebsmo(X, 6, 1, 4, 0.2, 2, Om)
    tau = full.rel_err[2] * 1.0001
    ref = g.grebsmo(X, 6, 1, 4, 0.2, 2, Om, tau=tau)
    gb = GreBsmo(dev(X), 6, dr=1, power=2, lam=0.2, seed=15)
    info = gb.solve(4, tau)
    assert info.stages == len(ref.rel_err) and info.rank == ref.ranks[-1]
    assert abs(info.rel_err_sq - ref.rel_err[-1]) <= 1e-12 * ref.rel_err[-1]
    gb.close()


def test_state_errors():
    from paper_1309_0302_amd.binding import GreBsmo, GodecError
    X, _ = problem(50, 40, 2, seed=16)
    gb = GreBsmo(dev(X), 2, dr=1, power=1, lam=0.1, seed=17)
    with pytest.raises(GodecError) as ei:
        gb.S()
    assert ei.value.status == 5
    gb.solve(2)
    with pytest.raises(GodecError) as ei:
        gb.stage(2)
    assert ei.value.status == 5
    gb.close()


def test_nonfinite_x_rejected():
    from paper_1309_0302_amd.binding import GreBsmo, GodecError
    X, _ = problem(40, 30, 2, seed=18)
    X[3, 4] = np.nan
    with pytest.raises(GodecError) as ei:
        GreBsmo(dev(X), 2)
    assert ei.value.status == 4
