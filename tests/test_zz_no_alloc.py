"""godec_solve_static, the entry point that allocates nothing: its results
must equal godec_solve's (the same kernels on a caller workspace) bit for
bit, on consecutive calls that share the library's device scratch, the
later ones on smaller problems (stale contents of the earlier call must not
leak into them); and oversized problems are rejected before any device work.
"""
import ctypes

import numpy as np
import pytest

from paper_1309_0302_amd import binding as b
from paper_1309_0302_amd import workloads as wl


def _bits(t):
    return np.ascontiguousarray(t.cpu().numpy()).view(np.uint8)


def _same(res_a, res_b):
    UL, VL, idx, val, info = res_a
    UL2, VL2, idx2, val2, info2 = res_b
    assert info["nnz"] == info2["nnz"] and info["rank_eff"] == info2["rank_eff"]
    for x, y in ((UL, UL2), (VL, VL2), (idx, idx2), (val, val2)):
        assert x.shape == y.shape
        assert np.array_equal(_bits(x), _bits(y))
    for key in ("rel_err_sq", "threshold", "sum_r2", "norm_x2"):
        assert np.float64(info[key]).tobytes() == np.float64(info2[key]).tobytes(), key


@pytest.mark.gpu
def test_static_equals_workspace_solve_on_consecutive_calls():
    torch = pytest.importorskip("torch")
    cases = [
        # (workload, prec, iterations): largest first, then smaller ones
        (wl.w2(), b.GODEC_PREC_NATIVE, 10),
        (wl.tiny(2000, 1500, 8, seed=31, dtype=np.float32), b.GODEC_PREC_BF16_REFINE, 4),
        (wl.w1(), b.GODEC_PREC_NATIVE, 20),
    ]
    for w, prec, iters in cases:
        m, n = w.X.shape
        print(f"\n[no-alloc] {m}x{n} {w.X.dtype} prec={prec} T={iters}", flush=True)
        dt = b.GODEC_F64 if w.X.dtype == np.float64 else b.GODEC_F32
        ws = b.godec_workspace_size(m, n, w.r, w.k, w.q, dt)
        assert ws <= b.GODEC_STATIC_SCRATCH_BYTES
        X = torch.from_numpy(w.X).cuda()
        opts, _ = b.make_opts(prec=prec, refine_iters=1)
        ref = b.godec_solve(X, w.r, w.k, w.q, 1234, iters, opts)
        got = b.godec_solve_static(X, w.r, w.k, w.q, 1234, iters, opts)
        torch.cuda.synchronize()
        _same(got, ref)
        del X


def test_static_rejects_oversized_problem_before_device_work():
    lib = b.load()
    opts, _ = b.make_opts()
    info = b.godec_info()
    # 10 000 x 10 000 FP32 needs far more than the scratch: rejected from the
    # size query alone (no device pointer is dereferenced)
    st = lib.godec_solve_static(None, b.GODEC_F32, 10000, 10000, 10000, 20, 2000000, 2, 1,
                                1, ctypes.byref(opts), None, None, None, None,
                                ctypes.byref(info))
    assert b.STATUS[st] == "GODEC_E_UNSUPPORTED"
    assert b"scratch" in lib.godec_last_error()
