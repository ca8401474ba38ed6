"""Precision forms against the FP64 oracle's own trajectory, and run-to-run
bit identity.

The per-step parity tests feed the oracle the GPU's own S_{t-1}; here each
GPU form runs T iterations from S_0 = 0 on its own, and the result is
compared with the oracle's own T-iteration run on the same X and A1
(Algorithm 1; the error measure of Sec. 5):
  * rel_L = ||L - L_o||_F / ||L_o||_F and the objective
    e = ||X - L - S||_F^2 / ||X||_F^2 against e_o (relative);
  * S on the common support (relative Frobenius), and the boundary swaps
    (entries in one support only) counted, each required to lie within the
    band 2 max|L - L_o| + |thr - thr_o| of the oracle's threshold: the S
    step is discontinuous, and a run whose L differs by rounding may land on
    a neighbouring fixed point that differs in entries at the threshold.
Cases: the 10 000 x 10 000 workload (r = 20, k = 2e6, q = 2) at T = 20 in
FP32 plain and in bf16 panels + one FP32 refinement iteration, and the same
recipe at 2000 x 2000 (k = 8e4) at T = 12.

Determinism: two runs of the same problem give bit-identical L factors, S
and objective (every cross-block sum is taken in a fixed order), for FP64,
FP32, the bf16 form and the batched form.
"""
import os
import sys

import numpy as np
import pytest
from conftest import oracle_a1

from oracle import godec_ref as g
from paper_1309_0302_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
from bench import trajectory_errors  # noqa: E402

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# Bars.  FP32 plain: 1e-5 on L, S (common support) and the objective, the
# FP32 tolerance of the method's parity bar (measured at 2000 x 2000:
# L 1.5e-7, S 6.6e-8, objective 2.3e-10, no swaps).
# The bf16 form: its iterations before the refinement compute L with a
# relative error near 2e-4, which flips S decisions of entries that close to
# the threshold; the S step keeps an entry's state (including it in S makes
# its next residual slightly larger, excluding it slightly smaller), so the
# run settles on a neighbouring fixed point whose support differs from the
# oracle's by such boundary entries, and the FP32 refinement keeps them.  L
# then differs from the oracle's L through those entries alone (the per-step
# parity after refinement is 1e-7).  Measured at 2000 x 2000: 64 swaps (8e-4
# of k, every one inside the band), L 2.7e-5, common-support S 1.1e-5,
# objective 3.1e-6.  Bars: objective 1e-5; L 5e-5; common-support S 3e-5;
# swaps at most 2e-3 of k and all inside the band.
FP32_BAR = 1e-5
BF16_OBJ_BAR = 1e-5
BF16_L_BAR = 5e-5
BF16_S_BAR = 3e-5
BF16_SWAP_FRAC = 2e-3


def run_gpu(X, w, prec, T, seed):
    from paper_1309_0302_amd.binding import GoDec
    print(f"\n[precision] {tuple(X.shape)} prec={prec} T={T}", flush=True)
    gd = GoDec(X, w.r, w.k, w.q, seed=seed, prec=prec, refine_iters=1)
    gd.step(T, T)
    info = gd.info()
    UL, VL = gd.factors()
    idx, val = gd.S()
    out = dict(UL=UL.double().cpu().numpy(), VL=VL.double().cpu().numpy(),
               idx=idx.cpu().numpy(), val=val.double().cpu().numpy(), info=info,
               A1=oracle_a1(gd))
    gd.close()
    return out


def check_forms(w, T, seed):
    from paper_1309_0302_amd.binding import GODEC_PREC_BF16_REFINE, GODEC_PREC_NATIVE
    X = torch.from_numpy(w.X).cuda()
    fp = run_gpu(X, w, GODEC_PREC_NATIVE, T, seed)
    bf = run_gpu(X, w, GODEC_PREC_BF16_REFINE, T, seed)
    del X
    torch.cuda.empty_cache()
    print(f"[precision] oracle: {T} iterations of {w.X.shape}", flush=True)
    tr = g.godec_brp(w.X.astype(np.float64), w.r, w.k, w.q, fp["A1"], T)
    res = {}
    for name, o in (("fp32", fp), ("bf16_refine", bf)):
        e = trajectory_errors(w.X, o["UL"], o["VL"], o["idx"], o["val"],
                              o["info"]["threshold"], tr.L, tr.S, tr.thresholds[-1])
        print(f"[precision] {name}: rel_L {e['rel_L']:.3e} rel_obj {e['rel_obj']:.3e} "
              f"rel_S_common {e['rel_S_common']:.3e} rel_S {e['rel_S']:.3e} "
              f"swaps {e['swaps']} (worst {e['swap_worst_dist']:.3e}, band "
              f"{e['swap_band']:.3e})", flush=True)
        res[name] = e
    for name, e in res.items():
        fp32 = name == "fp32"
        assert e["rel_obj"] <= (FP32_BAR if fp32 else BF16_OBJ_BAR), name
        assert e["rel_S_common"] <= (FP32_BAR if fp32 else BF16_S_BAR), name
        assert e["rel_L"] <= (FP32_BAR if fp32 else BF16_L_BAR), name
        assert e["swaps_within_band"], name
        if not fp32:
            assert e["swaps"] <= BF16_SWAP_FRAC * w.k, name
        # the support sizes agree (nnz = k) whatever the swaps
        assert e["common"] + e["swaps_gpu_only"] == w.k, name
    return res


def test_precision_forms_vs_oracle_2000():
    w = wl.w3(seed=2003, m=2000, n=2000)
    check_forms(w, 12, seed=2003)


def test_precision_forms_vs_oracle_full_size():
    w = wl.w3(seed=1003)
    check_forms(w, 20, seed=1003)


def solve_bits(X, r, k, q, prec, T, seed):
    from paper_1309_0302_amd.binding import GoDec
    gd = GoDec(X, r, k, q, seed=seed, prec=prec, refine_iters=1)
    gd.step(T, T)
    info = gd.info()
    UL, VL = gd.factors()
    idx, val = gd.S()
    out = (UL.cpu().numpy().copy(), VL.cpu().numpy().copy(), idx.cpu().numpy().copy(),
           val.cpu().numpy().copy(), np.float64(info["rel_err_sq"]),
           np.float64(info["sum_r2"]))
    gd.close()
    return out


@pytest.mark.parametrize("dtype,prec,shape,r,q", [
    (np.float64, 0, (700, 500), 6, 2),
    (np.float32, 0, (3001, 2003), 20, 2),
    (np.float32, 1, (3001, 2003), 20, 2),
])
def test_run_to_run_bit_identity(dtype, prec, shape, r, q):
    w = wl.tiny(shape[0], shape[1], r, seed=77, dtype=dtype)
    X = torch.from_numpy(w.X).cuda()
    print(f"\n[determinism] {shape} {np.dtype(dtype).name} prec={prec}", flush=True)
    a = solve_bits(X, r, w.k, q, prec, 5, 9)
    b = solve_bits(X, r, w.k, q, prec, 5, 9)
    for x, y in zip(a, b):
        assert np.array_equal(np.atleast_1d(np.asarray(x)).view(np.uint8), np.atleast_1d(np.asarray(y)).view(np.uint8))


def test_batch_run_to_run_bit_identity():
    from paper_1309_0302_amd.binding import GoDecBatch
    works = [wl.tiny(m, n, r, seed=80 + i, dtype=np.float32)
             for i, (m, n, r) in enumerate([(3000, 300, 4), (2100, 128, 8), (900, 400, 1)])]
    specs = [(torch.from_numpy(w.X).cuda(), w.r, w.k, 500 + i) for i, w in enumerate(works)]
    print("\n[determinism] batch of 3", flush=True)
    outs = []
    for _ in range(2):
        gb = GoDecBatch(specs, 1)
        gb.step(4)
        gb.synchronize()
        res = []
        for i in range(len(works)):
            info = gb.info(i)
            U, V = gb.factors(i)
            idx, val = gb.S(i)
            res.append((U.cpu().numpy().copy(), V.cpu().numpy().copy(),
                        np.sort(idx.cpu().numpy()), np.float64(info["rel_err_sq"]),
                        np.float64(info["sum_r2"]), np.float64(info["norm_x2"])))
        gb.close()
        outs.append(res)
    for ra, rb in zip(*outs):
        for x, y in zip(ra, rb):
            assert np.array_equal(np.atleast_1d(np.asarray(x)).view(np.uint8), np.atleast_1d(np.asarray(y)).view(np.uint8))
