"""Graph replay of the single-problem iteration (godec_set_graphs) against
direct launches, through the C ABI.

The same solve runs twice from the same inputs: once with every iteration
launched directly, once with the steady iterations replayed from recorded
HIP graphs.  After every step the factors, S and the objective must be the
same bits: replay runs the same kernels with the same arguments.  Between
the replayed steps the test does eager work of its own on the same stream
(a torch reduction, the accessors that launch and synchronise), as a caller
would.
"""
import numpy as np
import pytest

from paper_1309_0302_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def snapshot(gd):
    UL, VL = gd.factors()
    idx, val = gd.S()
    info = gd.info()
    return (UL.cpu().numpy().copy(), VL.cpu().numpy().copy(), idx.cpu().numpy().copy(),
            val.cpu().numpy().copy(), info["sum_r2"], info["nnz"], info["threshold"])


def same_bits(a, b):
    for x, y in zip(a, b):
        if isinstance(x, np.ndarray):
            assert x.shape == y.shape
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
        else:
            assert x == y


@pytest.mark.parametrize("dtype,prec,q,warm,redraw", [
    (np.float32, 0, 1, 0, 0),
    (np.float32, 1, 2, 0, 0),     # BF16 panels + FP32 refinement
    (np.float64, 0, 1, 0, 0),
    (np.float32, 0, 1, 1, 0),     # warm-started chains (a device copy in the graph)
    (np.float32, 1, 2, 0, 1),     # a new A1 per iteration, copied in ahead of each replay
])
def test_graph_replay_matches_direct_launches(dtype, prec, q, warm, redraw):
    from paper_1309_0302_amd.binding import GoDec
    w = wl.tiny(1500, 700, 6, rho=0.04, seed=31, dtype=dtype)
    X = torch.from_numpy(np.ascontiguousarray(w.X)).cuda()
    T = 9
    print(f"\n[graphs] dtype={np.dtype(dtype).name} prec={prec} q={q} warm={warm} "
          f"redraw={redraw} T={T}", flush=True)
    ref = []
    g0 = GoDec(X, w.r, w.k, q, seed=5, prec=prec, warm_start=warm,
               redraw_a1=redraw)
    try:
        for _ in range(T):
            g0.step(1, T)
            ref.append(snapshot(g0))
    finally:
        g0.close()
    g1 = GoDec(X, w.r, w.k, q, seed=5, prec=prec, warm_start=warm,
               redraw_a1=redraw)
    try:
        g1.graphs(True)
        for t in range(T):
            g1.step(1, T)
            # eager work of the caller between the replays
            _ = float(torch.sum(X[: 64].double()))
            torch.cuda.synchronize()
            same_bits(snapshot(g1), ref[t])
    finally:
        g1.close()


def test_graph_replay_multi_step_calls():
    """Several iterations per godec_step call, graphs recorded mid-solve."""
    from paper_1309_0302_amd.binding import GoDec
    w = wl.tiny(1200, 500, 4, rho=0.05, seed=32, dtype=np.float32)
    X = torch.from_numpy(np.ascontiguousarray(w.X)).cuda()
    g0 = GoDec(X, w.r, w.k, 1, seed=3)
    g0.step(2)
    g0.step(5)
    ref = snapshot(g0)
    g0.close()
    g1 = GoDec(X, w.r, w.k, 1, seed=3)
    g1.step(2)
    g1.graphs(True)
    g1.step(5)
    got = snapshot(g1)
    g1.close()
    same_bits(got, ref)
