"""GPU parity of the redrawn A1 (godec_opts.redraw_a1 = 1: iteration t draws
its own A1 from seed + t, as the MSE training of Algorithm 4 redraws it every
iteration) against the oracle's runs with a per-iteration A1, through the C
ABI.  The oracle draws every A1 with its own generator; the library's draws
are only checked against them, bit for bit.
"""
import numpy as np
import pytest

from oracle import godec_ref as g
from oracle.rng_ref import a1_gaussian
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


def draws(seed, n, r):
    return lambda t: a1_gaussian(seed + t, n, r)


@pytest.mark.parametrize("lstep", [0, 1])
def test_f64_w1_redrawn_trajectory(lstep):
    from paper_1309_0302_amd.binding import GoDec
    w = wl.w1()
    n = w.X.shape[1]
    print(f"\n[redraw] W1 FP64, lstep={lstep}, {w.iters} iterations", flush=True)
    gd = GoDec(dev(w.X), w.r, w.k, w.q, seed=w.seed, lstep=lstep, redraw_a1=1)
    try:
        gd.step(w.iters)
        ref = g.godec_brp(w.X, w.r, w.k, w.q, draws(w.seed, n, w.r), w.iters,
                          lstep="proj" if lstep else "root")
        # the A1 of the last iteration, as the oracle's generator draws it
        last = a1_gaussian(w.seed + w.iters - 1, n, w.r)
        assert np.array_equal(gd.A1().view(np.uint64), last.view(np.uint64))
        L = gd.L_dense().cpu().numpy()
        S = gpu_S(gd, w.X.shape)
        eL, eS = g.rel_fro(L, ref.L), g.rel_fro(S, ref.S)
        print(f"  L {eL:.2e}  S {eS:.2e}", flush=True)
        assert eL < 1e-10 and eS < 1e-10
    finally:
        gd.close()


def test_f64_redrawn_steps_against_the_oracle_per_step():
    """Every step from the GPU's own S: the oracle's step t with A1(t) on
    D = X - S_{t-1}, compared with the GPU's L_t (the root form's
    tolerance of 1e-10)."""
    from paper_1309_0302_amd.binding import GoDec
    w = wl.tiny(400, 300, 4, rho=0.05, seed=62, noise_std=1e-2)
    n = w.X.shape[1]
    print("\n[redraw] 400 x 300 FP64 q=1, per step", flush=True)
    gd = GoDec(dev(w.X), w.r, w.k, 1, seed=17, redraw_a1=1)
    try:
        S_prev = np.zeros_like(w.X)
        for t in range(6):
            gd.step(1)
            res = g.brp_power(w.X - S_prev, a1_gaussian(17 + t, n, w.r), 1)
            L = gd.L_dense().cpu().numpy()
            e = g.rel_fro(L, res.L)
            print(f"  step {t}: L {e:.2e}", flush=True)
            assert e < 1e-10
            S_prev = gpu_S(gd, w.X.shape)
    finally:
        gd.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_f32_redrawn_run_reaches_the_oracle(prec):
    """FP32 panels (1e-5) and BF16 panels + one FP32 refinement iteration
    against the FP64 oracle's redrawn run.  The bf16 iterations before the
    refinement can flip S decisions of entries at the threshold, and the run
    keeps them, so its L bar is that of the bf16 form against the oracle's
    own run (5e-5), not the per-step one."""
    from paper_1309_0302_amd.binding import GoDec
    w = wl.tiny(1000, 700, 5, rho=0.04, seed=63, dtype=np.float32, noise_std=1e-3)
    n = w.X.shape[1]
    T = 12
    print(f"\n[redraw] 1000 x 700 FP32 prec={prec} q=1, {T} iterations", flush=True)
    gd = GoDec(dev(w.X), w.r, w.k, 1, seed=5, prec=prec, redraw_a1=1)
    try:
        gd.step(T, T)
        ref = g.godec_brp(w.X.astype(np.float64), w.r, w.k, 1, draws(5, n, w.r), T)
        L = gd.L_dense().cpu().numpy().astype(np.float64)
        eL = g.rel_fro(L, ref.L)
        print(f"  L vs oracle {eL:.2e}", flush=True)
        assert eL < (1e-5 if prec == 0 else 5e-5)
    finally:
        gd.close()


def test_redrawn_first_step_equals_the_fixed_one_and_calls_compose():
    """Iteration 0 uses the seed's own draw (the default mode's A1), and the
    iteration count that keys the draws runs on across godec_step calls."""
    from paper_1309_0302_amd.binding import GoDec
    w = wl.tiny(300, 200, 4, seed=64, dtype=np.float32)
    X = dev(w.X)
    a = GoDec(X, 4, w.k, 1, seed=3, redraw_a1=1)
    b = GoDec(X, 4, w.k, 1, seed=3)
    c = GoDec(X, 4, w.k, 1, seed=3, redraw_a1=1)
    try:
        a.step(1)
        b.step(1)
        assert torch.equal(a.L_dense(), b.L_dense())
        a.step(2)
        a.step(4)
        c.step(7)
        assert torch.equal(a.L_dense(), c.L_dense())
        ia, ic = a.S(), c.S()
        assert torch.equal(ia[0], ic[0]) and torch.equal(ia[1], ic[1])
        b.step(6)
        assert not torch.equal(a.L_dense(), b.L_dense())
    finally:
        a.close()
        b.close()
        c.close()


def test_static_entry_rejects_redraw():
    from paper_1309_0302_amd import binding as bd
    w = wl.tiny(120, 100, 3, seed=65, dtype=np.float32)
    o, _ = bd.make_opts(redraw_a1=1)
    with pytest.raises(bd.GodecError) as ei:
        bd.godec_solve_static(dev(w.X), 3, w.k, 1, 2, 3, opts=o)
    assert "redraw_a1" in str(ei.value)


def test_f64_completion_with_redrawn_a1():
    """The fixed-support S update with a new A1 per iteration against the
    completion oracle's redrawn run (no discrete decisions on a fixed
    support, so the FP64 bar is 1e-10 over the whole run), and exact
    completion of a rank-3 matrix."""
    from oracle import completion_ref as cr
    from paper_1309_0302_amd.binding import GoDec
    rng = np.random.default_rng(66)
    m, n, r = 150, 110, 3
    X0 = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    miss = np.sort(rng.choice(m * n, size=int(0.3 * m * n), replace=False))
    for noise, T in ((1e-2, 10), (0.0, 100)):
        X = X0 + noise * np.random.default_rng(67).standard_normal((m, n))
        X.flat[miss] = 0.0
        sup = torch.from_numpy(miss.astype(np.int64)).cuda()
        print(f"\n[redraw] completion 150 x 110 FP64 noise={noise} T={T}", flush=True)
        gd = GoDec(dev(X), r, int(miss.size), 1, seed=21, support=sup, redraw_a1=1)
        try:
            gd.step(T)
            L = gd.L_dense().cpu().numpy()
            ref = cr.godec_completion(X, r, 1, draws(21, n, r), miss, T)
            eL = g.rel_fro(L, ref.L)
            print(f"  L vs oracle {eL:.2e}", flush=True)
            assert eL < 1e-10
            if noise == 0.0:
                assert g.rel_fro(L, X0) < 1e-10
        finally:
            gd.close()


def test_solve_tol_with_redrawn_a1():
    """godec_solve_tol with a new A1 per iteration stops where the oracle's
    redrawn run first meets the loop test, with the same factors as that
    many steps of a context (draws are staged for max_iters iterations, so
    the solve ends with unused draws in flight)."""
    from paper_1309_0302_amd import binding as bd
    w = wl.tiny(300, 200, 5, seed=22, dtype=np.float64)
    n = w.X.shape[1]
    tr = g.godec_brp(w.X, 5, w.k, 1, draws(99, n, 5), 12)
    errs = np.asarray(tr.rel_err_sq)
    assert errs[2] > 1.01 * errs[3]
    eps = float(np.sqrt(errs[2] * errs[3]))
    expect = int(np.argmax(errs <= eps)) + 1
    print(f"\n[redraw] solve_tol: errors {errs[:6]}, eps {eps:.3e}, expect {expect}", flush=True)
    o, _ = bd.make_opts(redraw_a1=1)
    UL, VL, _, _, info = bd.godec_solve_tol(dev(w.X), 5, w.k, 1, 99, 12, eps, o)
    assert info["iters"] == expect
    gd = bd.GoDec(dev(w.X), 5, w.k, 1, seed=99, redraw_a1=1)
    try:
        gd.step(expect)
        U2, _ = gd.factors()
        assert np.array_equal(UL.cpu().numpy(), U2.cpu().numpy())
    finally:
        gd.close()
