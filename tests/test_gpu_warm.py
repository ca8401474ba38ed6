"""GPU parity of the warm-started power chains (godec_opts.warm_start = 1:
every chain after the first starts from the previous iteration's Q2 instead
of A1; a variant outside the paper) against the oracle's own warm-started
runs, through the C ABI.  The oracle never takes the GPU's Q2: it carries
its own right factor from step to step.
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


@pytest.mark.parametrize("lstep", [0, 1])
def test_f64_w1_warm_trajectory(lstep):
    from paper_1309_0302_amd.binding import GoDec
    w = wl.w1()
    print(f"\n[warm] W1 FP64, lstep={lstep}, 20 iterations", flush=True)
    gd = GoDec(dev(w.X), w.r, w.k, w.q, seed=w.seed, lstep=lstep, warm_start=1)
    gd.step(w.iters)
    ref = g.godec_brp(w.X, w.r, w.k, w.q, oracle_a1(gd), w.iters, warm=True,
                      lstep="proj" if lstep else "root")
    L = gd.L_dense().cpu().numpy()
    S = gpu_S(gd, w.X.shape)
    eL, eS = g.rel_fro(L, ref.L), g.rel_fro(S, ref.S)
    print(f"  L {eL:.2e}  S {eS:.2e}", flush=True)
    assert eL < 1e-10 and eS < 1e-10
    gd.close()


@pytest.mark.parametrize("q", [0, 1])
def test_f32_warm_reaches_the_oracle_fixed_point(q):
    from paper_1309_0302_amd.binding import GoDec
    w = wl.tiny(1000, 700, 5, rho=0.04, seed=31 + q, dtype=np.float32, noise_std=1e-3)
    print(f"\n[warm] 1000 x 700 FP32 q={q}, 15 iterations", flush=True)
    gd = GoDec(dev(w.X), w.r, w.k, q, seed=5, warm_start=1)
    gd.step(15)
    ref = g.godec_brp(w.X.astype(np.float64), w.r, w.k, q, oracle_a1(gd), 15, warm=True)
    L = gd.L_dense().cpu().numpy().astype(np.float64)
    eL = g.rel_fro(L, ref.L)
    e0 = g.rel_fro(L, w.L0)
    print(f"  L vs oracle {eL:.2e}, vs planted L0 {e0:.2e}", flush=True)
    assert eL < 1e-5
    gd.close()


def test_warm_first_step_equals_cold():
    from paper_1309_0302_amd.binding import GoDec
    w = wl.tiny(300, 200, 4, seed=41, dtype=np.float32)
    a = GoDec(dev(w.X), 4, w.k, 1, seed=3, warm_start=1)
    b = GoDec(dev(w.X), 4, w.k, 1, seed=3)
    a.step(1)
    b.step(1)
    assert torch.equal(a.L_dense(), b.L_dense())
    a.close()
    b.close()


def test_f64_warm_start_after_a_rank_drop():
    """X of rank 3 with r = 5: the first iteration drops the rank (the root
    form's rank check) and the warm chains continue on the kept directions,
    as the oracle's warm run does."""
    from paper_1309_0302_amd.binding import GoDec
    rng = np.random.default_rng(52)
    X = rng.standard_normal((150, 3)) @ rng.standard_normal((3, 110))
    print("\n[warm] rank-3 150 x 110 FP64 with r = 5, 4 iterations", flush=True)
    gd = GoDec(dev(X), 5, 0, 1, seed=4, warm_start=1)
    gd.step(4)
    ref = g.godec_brp(X, 5, 0, 1, oracle_a1(gd), 4, warm=True)
    L = gd.L_dense().cpu().numpy()
    info = gd.info()
    print(f"  rank_eff {info['rank_eff']} (oracle {ref.r_eff}), L vs oracle "
          f"{g.rel_fro(L, ref.L):.2e}", flush=True)
    assert info["rank_eff"] == ref.r_eff == 3
    assert g.rel_fro(L, ref.L) < 1e-10 and g.rel_fro(L, X) < 1e-10
    gd.close()
