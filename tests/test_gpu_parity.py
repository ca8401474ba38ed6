"""GPU parity of libgodec against the FP64 oracle, through the C ABI.

Per-step parity: before every GPU iteration the GPU's own S_{t-1} is read
back, the oracle runs the same low-rank step on D = X - S_{t-1} with the same
A1, and the GPU's L_t must match within the dtype's tolerance (relative
Frobenius, non-squared: 1e-10 FP64, 1e-5 FP32, 2e-3 BF16 before refinement,
1e-5 after).  The support of S_t must equal, bit for bit, the oracle's
hard threshold applied to the GPU's own residual (the decision is taken in
the GPU's precision on both sides), and the values must be the residual's.
"""
import numpy as np
import pytest
from conftest import oracle_a1

from oracle import godec_ref as g
from paper_1309_0302_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(X):
    return torch.from_numpy(np.ascontiguousarray(X)).cuda()


def gpu_S(gd, shape):
    idx, val = gd.S()
    S = np.zeros(int(np.prod(shape)), dtype=np.float64)
    S[idx.cpu().numpy()] = val.cpu().numpy().astype(np.float64)
    return S.reshape(shape)


def check_support(gd, k):
    """S_t == hard threshold of the GPU residual, bitwise."""
    R = gd.residual().cpu().numpy()
    ridx, rval = g.hard_threshold(R, k)
    sidx, sval = gd.S()
    sidx = sidx.cpu().numpy()
    sval = sval.cpu().numpy()
    assert np.array_equal(sidx, ridx), (sidx.size, ridx.size)
    assert np.array_equal(sval.view(np.uint8), rval.astype(sval.dtype).view(np.uint8))
    return sidx


def per_step(X, r, k, q, iters, tol, *, seed=7, prec=0, refine_iters=1,
             total=0, tols=None, rank_tol=None):
    from paper_1309_0302_amd.binding import GoDec
    print(f"\n[per_step] shape={X.shape} dtype={X.dtype} r={r} k={k} q={q} "
          f"iters={iters} prec={prec}", flush=True)
    gd = GoDec(dev(X), r, k, q, seed=seed, prec=prec, refine_iters=refine_iters,
               rank_tol=rank_tol or 0.0)
    A1 = oracle_a1(gd)
    X64 = X.astype(np.float64)
    errs = []
    try:
        for t in range(iters):
            S_prev = gpu_S(gd, X.shape)
            r_eff = gd.info()["rank_eff"]
            gd.step(1, total)
            torch.cuda.synchronize()
            ref = g.brp_power(X64 - S_prev, A1[:, :r_eff], q, rank_tol)
            L = gd.L_dense().cpu().numpy().astype(np.float64)
            err = g.rel_fro(L, ref.L)
            errs.append(err)
            lim = tols[t] if tols is not None else tol
            assert err <= lim, (t, err, lim)
            assert gd.info()["rank_eff"] == ref.r_eff
            check_support(gd, k)
        info = gd.info()
        assert info["nnz"] <= k
        return gd, errs
    finally:
        pass


# ---------------------------------------------------------------------------
# FP64
# ---------------------------------------------------------------------------

def test_f64_w1_per_step():
    w = wl.w1()
    per_step(w.X, w.r, w.k, w.q, 4, 1e-10, seed=w.seed)


def test_f64_w1_trajectory_20_iterations():
    from paper_1309_0302_amd.binding import GoDec
    w = wl.w1()
    gd = GoDec(dev(w.X), w.r, w.k, w.q, seed=w.seed)
    gd.step(w.iters)
    ref = g.godec_brp(w.X, w.r, w.k, w.q, oracle_a1(gd), w.iters)
    L = gd.L_dense().cpu().numpy()
    S = gpu_S(gd, w.X.shape)
    assert g.rel_fro(L, ref.L) < 1e-10
    assert np.array_equal(np.flatnonzero(S), np.flatnonzero(ref.S))
    assert g.rel_fro(S, ref.S) < 1e-10
    info = gd.info()
    assert info["nnz"] == w.k
    assert abs(info["rel_err_sq"] - ref.rel_err_sq[-1]) <= 1e-8 * ref.rel_err_sq[-1]


@pytest.mark.parametrize("m,n,r,q", [(300, 200, 5, 2), (200, 300, 3, 1),
                                     (131, 77, 12, 0), (97, 413, 20, 1)])
def test_f64_shapes_per_step(m, n, r, q):
    w = wl.tiny(m, n, r, seed=m + n, dtype=np.float64)
    per_step(w.X, r, w.k, q, 2, 1e-10)


# ---------------------------------------------------------------------------
# FP32: shapes spanning several tiles and ragged tails, every panel width
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,r,q", [
    (300, 200, 5, 2), (200, 300, 3, 1), (517, 129, 8, 0), (1000, 37, 13, 1),
    (64, 1500, 20, 2), (257, 255, 32, 1), (33, 17, 1, 0), (2100, 300, 2, 1),
    (1030, 1100, 16, 2), (700, 257, 24, 1), (300, 300, 4, 3),
])
def test_f32_shapes_per_step(m, n, r, q):
    w = wl.tiny(m, n, r, seed=3 * m + n, dtype=np.float32)
    per_step(w.X, r, w.k, q, 3, 1e-5)


def test_f32_w2_video_per_step():
    w = wl.w2()
    per_step(w.X, w.r, w.k, w.q, 3, 1e-5, seed=w.seed)


def test_f32_w2_video_trajectory():
    from paper_1309_0302_amd.binding import GoDec
    w = wl.w2()
    gd = GoDec(dev(w.X), w.r, w.k, w.q, seed=w.seed)
    gd.step(w.iters)
    ref = g.godec_brp(w.X.astype(np.float64), w.r, w.k, w.q, oracle_a1(gd), w.iters)
    L = gd.L_dense().cpu().numpy().astype(np.float64)
    S = gpu_S(gd, w.X.shape)
    errL = g.rel_fro(L, ref.L)
    sup_g, sup_o = np.flatnonzero(S), np.flatnonzero(ref.S)
    swaps = np.setxor1d(sup_g, sup_o).size
    common = np.intersect1d(sup_g, sup_o)
    errS = np.linalg.norm(S.flat[common] - ref.S.flat[common]) / np.linalg.norm(ref.S.flat[common])
    print(f"\n[w2 trajectory] L err {errL:.3e} common-support S err {errS:.3e} swaps {swaps}")
    assert errL < 1e-5
    assert errS < 1e-5
    assert swaps <= 1e-4 * w.k


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------

def test_k_zero_keeps_s_empty():
    w = wl.tiny(120, 90, 4, seed=1, dtype=np.float32)
    gd, _ = per_step(w.X, 4, 0, 1, 2, 1e-5)
    assert gd.info()["nnz"] == 0


def test_k_all_entries():
    w = wl.tiny(60, 50, 3, seed=2, dtype=np.float32)
    gd, _ = per_step(w.X, 3, 60 * 50, 1, 2, 1e-5)
    R = gd.residual().cpu().numpy()
    assert gd.info()["nnz"] == np.count_nonzero(R)


def test_tie_heavy_integer_matrix_f32():
    """Many exact ties at the threshold: the index tie-break decides."""
    rng = np.random.default_rng(5)
    X = rng.integers(-2, 3, size=(150, 140)).astype(np.float32)
    X[:, :70] = 1.0               # a constant block makes L nearly exact there
    per_step(X, 2, 3000, 1, 3, 1e-5)


def test_tie_heavy_f64_many_ties():
    rng = np.random.default_rng(6)
    X = np.where(rng.random((200, 180)) < 0.5, 1.0, 0.0)
    per_step(X, 1, 5000, 0, 2, 1e-10)


def test_zero_residuals_never_selected():
    rng = np.random.default_rng(8)
    U, V = rng.standard_normal((80, 2)), rng.standard_normal((60, 2))
    X = (U @ V.T)
    X[:5, :5] += 10.0
    gd, _ = per_step(X, 2, 2000, 1, 3, 1e-10)
    assert gd.info()["nnz"] <= 2000


def test_rank_deficient_input_drops_rank():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((150, 3)) @ rng.standard_normal((3, 120))
    gd, _ = per_step(X, 6, 10, 2, 3, 1e-9)
    assert gd.info()["rank_eff"] == 3
    assert gd.info()["flags"] & 2


def test_rank_deficient_f32():
    rng = np.random.default_rng(10)
    X = (rng.standard_normal((300, 2)) @ rng.standard_normal((2, 250))).astype(np.float32)
    gd, _ = per_step(X, 5, 20, 1, 2, 1e-5)
    assert gd.info()["rank_eff"] == 2


def test_nan_in_x_rejected():
    from paper_1309_0302_amd.binding import GoDec, GodecError
    X = np.ones((40, 30), dtype=np.float32)
    X[3, 4] = np.nan
    with pytest.raises(GodecError) as ei:
        GoDec(dev(X), 2, 10, 1)
    assert ei.value.status == 4


def test_strided_x_leading_dimension():
    """X with ldx > n (a column slice of a wider buffer)."""
    from paper_1309_0302_amd.binding import GoDec
    w = wl.tiny(200, 150, 4, seed=12, dtype=np.float32)
    big = np.zeros((200, 181), dtype=np.float32)
    big[:, :150] = w.X
    Xd = dev(big)[:, :150]
    gd = GoDec(Xd, 4, w.k, 1, seed=3)
    gd.step(2)
    gd2 = GoDec(dev(w.X), 4, w.k, 1, seed=3)
    gd2.step(2)
    a = gd.L_dense().cpu().numpy()
    c = gd2.L_dense().cpu().numpy()
    assert np.array_equal(a, c)


def test_seeded_a1_matches_oracle_generator():
    from oracle.rng_ref import a1_gaussian
    from paper_1309_0302_amd.binding import GoDec
    w = wl.tiny(50, 40, 3, seed=1, dtype=np.float32)
    gd = GoDec(dev(w.X), 3, 20, 1, seed=424242)
    assert np.array_equal(gd.A1(), a1_gaussian(424242, 40, 3))


def test_solve_entry_point_matches_step_path():
    from paper_1309_0302_amd import binding as b
    w = wl.tiny(300, 200, 5, seed=21, dtype=np.float32)
    UL, VL, sidx, sval, info = b.godec_solve(dev(w.X), 5, w.k, 1, 99, 4)
    gd = b.GoDec(dev(w.X), 5, w.k, 1, seed=99)
    gd.step(4)
    U2, V2 = gd.factors()
    assert np.array_equal(UL.cpu().numpy(), U2.cpu().numpy())
    i2, v2 = gd.S()
    assert np.array_equal(sidx.cpu().numpy(), i2.cpu().numpy())
    assert info["iters"] == 4


def test_solve_tol_stops_at_the_loop_test():
    """godec_solve_tol stops after the first iteration whose relative error is
    <= eps (Algorithm 1's loop test), with the same result as that many
    plain steps; the oracle's error sequence says where that is."""
    from paper_1309_0302_amd import binding as b
    from oracle.rng_ref import a1_gaussian
    w = wl.tiny(300, 200, 5, seed=22, dtype=np.float64)
    A1 = a1_gaussian(99, 200, 5)
    tr = g.godec_brp(w.X, 5, w.k, 1, A1, 12)
    errs = np.asarray(tr.rel_err_sq)
    assert errs[2] > 1.01 * errs[3]                # a clear step to stop at
    eps = float(np.sqrt(errs[2] * errs[3]))       # between the 3rd and 4th errors
    expect = int(np.argmax(errs <= eps)) + 1
    print(f"\n[solve_tol] errors {errs[:6]}, eps {eps:.3e}, expect {expect}", flush=True)
    UL, VL, sidx, sval, info = b.godec_solve_tol(dev(w.X), 5, w.k, 1, 99, 12, eps)
    assert info["iters"] == expect
    assert info["rel_err_sq"] <= eps
    gd = b.GoDec(dev(w.X), 5, w.k, 1, seed=99)
    gd.step(expect)
    U2, V2 = gd.factors()
    assert np.array_equal(UL.cpu().numpy(), U2.cpu().numpy())
    # eps = 0 runs all max_iters; bf16 + refinement ends with the refinement
    _, _, _, _, info0 = b.godec_solve_tol(dev(w.X), 5, w.k, 1, 99, 5, 0.0)
    assert info0["iters"] == 5
    wf = wl.tiny(600, 400, 4, seed=23, dtype=np.float32)
    opts, _ = b.make_opts(prec=1, refine_iters=1)
    _, _, _, _, inf1 = b.godec_solve_tol(dev(wf.X), 4, wf.k, 1, 7, 6, 1e30, opts)
    assert inf1["iters"] == 2                      # one tested iteration + one refinement


# ---------------------------------------------------------------------------
# Mixed precision: bf16 panels with FP32 accumulation and FP32 refinement
# ---------------------------------------------------------------------------

def test_bf16_then_refine_per_step():
    w = wl.tiny(2000, 1500, 8, seed=31, dtype=np.float32, factor_std=0.5)
    # three iterations, the last one refined
    per_step(w.X, 8, w.k, 2, 3, None, prec=1, refine_iters=1, total=3,
             tols=[2e-3, 2e-3, 1e-5])
