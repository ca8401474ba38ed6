"""Parity at the full 10000 x 10000 workload, in the configuration the
benchmark times (same shape, so the library picks the same launch grids).

Per step: the oracle runs the low-rank step of Algorithm 1 on D = X - S_{t-1}
built from the GPU's own S_{t-1} and the GPU's A1; L_t is compared through
its factors (relative Frobenius norm, non-squared).  Tolerances: 2e-3 for the
BF16 iterations, 1e-5 for the FP32 refinement iteration and for FP32 plain.
The support of S_t must equal, bit for bit, the hard threshold (Eq. 4, ties
by row-major index) of the GPU's own residual, and its values must be the
residual's.
"""
import numpy as np
import pytest
from conftest import oracle_a1

from oracle import godec_ref as g
from paper_1309_0302_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def w3():
    print("\n[fullsize] generating the 10000 x 10000 workload", flush=True)
    return wl.w3()


def _step_and_check(gd, X64, q, k, tol, total, A1):
    idx, val = gd.S()
    S = np.zeros(X64.size)
    S[idx.cpu().numpy()] = val.cpu().numpy().astype(np.float64)
    r_eff = gd.info()["rank_eff"]
    gd.step(1, total)
    torch.cuda.synchronize()
    D = X64 - S.reshape(X64.shape)
    del S
    ref = g.brp_power(D, A1[:, :r_eff], q)
    del D
    UL, VL = gd.factors()
    UL = UL.cpu().numpy().astype(np.float64)
    VL = VL.cpu().numpy().astype(np.float64)
    err = g.rel_fro_factors(UL, VL, ref.left, ref.right)
    print(f"[fullsize] step {gd.info()['iters']}: rel L err {err:.3e} (tol {tol:.0e})",
          flush=True)
    assert err <= tol, (err, tol)
    assert gd.info()["rank_eff"] == ref.r_eff
    # support: bitwise against the hard threshold of the GPU residual
    R = gd.residual().cpu().numpy()
    ridx, rval = g.hard_threshold(R, k)
    del R
    sidx, sval = gd.S()
    sidx = sidx.cpu().numpy()
    sval = sval.cpu().numpy()
    assert np.array_equal(sidx, ridx), (sidx.size, ridx.size)
    assert np.array_equal(sval.view(np.uint32), rval.astype(np.float32).view(np.uint32))


def test_w3_bf16_refine_per_step(w3):
    from paper_1309_0302_amd.binding import GODEC_PREC_BF16_REFINE, GoDec
    X = torch.from_numpy(w3.X).cuda()
    gd = GoDec(X, w3.r, w3.k, w3.q, seed=w3.seed, prec=GODEC_PREC_BF16_REFINE,
               refine_iters=1)
    X64 = w3.X.astype(np.float64)
    A1 = oracle_a1(gd)
    total = 3
    for t, tol in enumerate((2e-3, 2e-3, 1e-5)):
        print(f"[fullsize] bf16+refine iteration {t} of {total}", flush=True)
        _step_and_check(gd, X64, w3.q, w3.k, tol, total, A1)
    gd.close()


def test_w3_fp32_plain_per_step(w3):
    from paper_1309_0302_amd.binding import GoDec
    X = torch.from_numpy(w3.X).cuda()
    gd = GoDec(X, w3.r, w3.k, w3.q, seed=w3.seed)
    X64 = w3.X.astype(np.float64)
    A1 = oracle_a1(gd)
    for t in range(2):
        print(f"[fullsize] fp32 iteration {t}", flush=True)
        _step_and_check(gd, X64, w3.q, w3.k, 1e-5, 0, A1)
    gd.close()
