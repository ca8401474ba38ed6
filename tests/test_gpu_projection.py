"""GPU parity of the projection form of the L update (godec_opts.lstep = 1:
L = (X - S) P_{Y2}, the form App. II Thm. 4 bounds) against the FP64
oracle's brp_projection, through the C ABI.

Per step, on the GPU's own S_{t-1} and the oracle's own A1: L_t within
1e-10 (FP64), 1e-5 (FP32), 2e-3 for BF16 panels before the FP32 refinement
and 1e-5 after it (the bars of the root form); the support of S_t bit-exact
against a CPU top-k of the GPU's own residual.  Trajectory: 20 FP64
iterations of the 500 x 500 workload against the oracle's own run.
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
    S = np.zeros(int(np.prod(shape)))
    S[idx.cpu().numpy()] = val.cpu().numpy().astype(np.float64)
    return S.reshape(shape)


def per_step(X, r, k, q, tols, prec=0, seed=7):
    from paper_1309_0302_amd.binding import GoDec
    print(f"\n[proj] shape={X.shape} dtype={X.dtype} r={r} k={k} q={q} prec={prec}", flush=True)
    gd = GoDec(dev(X), r, k, q, seed=seed, prec=prec, lstep=1)
    A1 = oracle_a1(gd)
    X64 = X.astype(np.float64)
    errs = []
    for t, tol in enumerate(tols):
        S_prev = gpu_S(gd, X.shape)
        gd.step(1, len(tols))
        torch.cuda.synchronize()
        ref = g.brp_projection(X64 - S_prev, A1, q)
        L = gd.L_dense().cpu().numpy().astype(np.float64)
        err = g.rel_fro(L, ref.L)
        errs.append(err)
        R = gd.residual().cpu().numpy()
        ridx, rval = g.hard_threshold(R, k)
        sidx, sval = gd.S()
        assert np.array_equal(sidx.cpu().numpy(), ridx), t
        assert np.array_equal(sval.cpu().numpy().view(np.uint8),
                              rval.astype(sval.cpu().numpy().dtype).view(np.uint8)), t
        assert err <= tol, (t, err, tol)
    print("  per-step L errors: " + " ".join(f"{e:.2e}" for e in errs), flush=True)
    gd.close()


def test_f64_w1_per_step():
    w = wl.w1()
    per_step(w.X, w.r, w.k, w.q, [1e-10] * 5)


@pytest.mark.parametrize("m,n,r,q", [(2000, 1500, 8, 1), (1037, 777, 5, 2), (300, 700, 20, 0)])
def test_f32_per_step(m, n, r, q):
    w = wl.tiny(m, n, r, rho=0.04, seed=m + n, dtype=np.float32, noise_std=1e-2)
    per_step(w.X, r, w.k, q, [1e-5] * 3)


def test_bf16_refine_per_step():
    from paper_1309_0302_amd.binding import GODEC_PREC_BF16_REFINE
    w = wl.tiny(2000, 1500, 8, rho=0.04, seed=9, dtype=np.float32, noise_std=1e-2)
    per_step(w.X, 8, w.k, 2, [2e-3, 2e-3, 1e-5], prec=GODEC_PREC_BF16_REFINE)


def test_f64_w1_trajectory():
    from paper_1309_0302_amd.binding import GoDec
    w = wl.w1()
    gd = GoDec(dev(w.X), w.r, w.k, w.q, seed=w.seed, lstep=1)
    gd.step(w.iters)
    ref = g.godec_brp(w.X, w.r, w.k, w.q, oracle_a1(gd), w.iters, lstep="proj")
    L = gd.L_dense().cpu().numpy()
    S = gpu_S(gd, w.X.shape)
    eL, eS = g.rel_fro(L, ref.L), g.rel_fro(S, ref.S)
    print(f"\n[proj] W1 20 iterations: L {eL:.2e}, S {eS:.2e}", flush=True)
    assert eL < 1e-10 and eS < 1e-10
    assert abs(gd.info()["rel_err_sq"] - ref.rel_err_sq[-1]) <= 1e-9 * ref.rel_err_sq[-1]
    gd.close()


def test_f64_rank_deficient_x():
    """X of rank 2 with r = 4: the dependent directions of Q2 come out as zero
    columns on the GPU, and L = X exactly, as the oracle's projection gives."""
    from paper_1309_0302_amd.binding import GoDec
    rng = np.random.default_rng(51)
    X = rng.standard_normal((120, 2)) @ rng.standard_normal((2, 90))
    print("\n[proj] rank-2 120 x 90 FP64 with r = 4", flush=True)
    gd = GoDec(dev(X), 4, 0, 1, seed=3, lstep=1)
    gd.step(2)
    L = gd.L_dense().cpu().numpy()
    ref = g.brp_projection(X, oracle_a1(gd), 1)
    print(f"  L vs X {g.rel_fro(L, X):.2e}, vs oracle {g.rel_fro(L, ref.L):.2e}", flush=True)
    assert g.rel_fro(L, X) < 1e-12 and g.rel_fro(L, ref.L) < 1e-12
    assert np.all(np.isfinite(L))
    gd.close()
