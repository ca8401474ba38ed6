"""GPU parity of MSE training (Sec. 4.2.1, Algorithm 4) against the FP64
oracle (oracle/mse_ref.py), through the C ABI.

Per step: the oracle's iteration t runs from the GPU's own state after
iteration t - 1 (every label's L^i = U_i V_i^T and S) with the same A1
draws; every label's L^i and the objective must match within the dtype's
tolerance (1e-10 FP64, 1e-5 FP32), and the support of S must equal, bit for
bit, a CPU top-K of the residual the GPU selected from (E + S, where E is the
GPU's X - sum L - S).  Trajectories: the GPU's T iterations against the
oracle's own T iterations.  Edge cases: an empty label, a sample without
labels, a label with fewer rows than its rank, K = 0, disjoint labels (one
sweep recovers every block), bit identity from run to run, and the
65 536 x 512, 32-label workload at full size.
"""
import numpy as np
import pytest

from oracle import godec_ref as g
from oracle import mse_ref as M
from paper_1309_0302_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def gpu_state(gm):
    Ls = []
    for i in range(gm.k):
        U, V = gm.factors(i)
        Ls.append(U.double().cpu().numpy() @ V.double().cpu().numpy().T)
    idx, val = gm.S()
    S = np.zeros(gm.n * gm.p)
    S[idx.cpu().numpy()] = val.double().cpu().numpy()
    return Ls, S.reshape(gm.n, gm.p), idx.cpu().numpy(), val.cpu().numpy()


def check_support(gm, idx, val):
    """The support equals a CPU top-K of the residual the GPU selected from,
    in the GPU's own precision; S holds that residual there."""
    E = gm.residual().cpu().numpy()
    R = E.copy()
    R.ravel()[idx] = val            # E is exactly 0 on the support
    ref_idx, ref_val = g.hard_threshold(R, gm.K)
    assert np.array_equal(np.sort(idx), ref_idx)
    order = np.argsort(idx)
    assert np.array_equal(val[order].view(np.uint8), ref_val.view(np.uint8))
    assert np.all(E.ravel()[idx] == 0)


def per_step(w, dtype, T, tol, label=""):
    from paper_1309_0302_amd.binding import GoDecMSE
    Xn = np.ascontiguousarray(w.X.astype(dtype))
    X = torch.from_numpy(Xn).cuda()
    print(f"\n[mse] per step {label} {Xn.shape} {np.dtype(dtype).name} k={len(w.labels)} "
          f"K={w.K} T={T}", flush=True)
    gm = GoDecMSE(X, w.labels, w.ranks, w.K, seed=w.seed)
    Xo = Xn.astype(np.float64)
    state = None
    worst = 0.0
    for t in range(T):
        ref = M.mse_train(Xo, w.labels, w.ranks, w.K, w.seed, 1, state=state, t0=t)
        gm.step(1)
        Ls, S, idx, val = gpu_state(gm)
        for i in range(len(w.labels)):
            e = rel(Ls[i], ref.Ls[i])
            worst = max(worst, e)
            assert e < tol, (t, i, e)
        check_support(gm, idx, val)
        info = gm.info()
        assert info["nnz"] == len(idx)
        e_obj = abs(info["rel_err_sq"] - ref.rel_err_sq[-1]) / max(ref.rel_err_sq[-1], 1e-300)
        assert e_obj < tol, (t, e_obj)
        state = (Ls, S)
    print(f"[mse] worst per-step L error {worst:.2e}", flush=True)
    gm.close()
    return worst


def test_per_step_fp64_mse1():
    per_step(wl.mse1(), np.float64, 6, 1e-10, "mse1")


def test_per_step_fp32_mse1():
    per_step(wl.mse1(), np.float32, 6, 1e-5, "mse1")


def test_trajectory_fp64_mse1():
    from paper_1309_0302_amd.binding import GoDecMSE
    w = wl.mse1()
    X = torch.from_numpy(w.X).cuda()
    print("\n[mse] trajectory mse1 FP64 T=10", flush=True)
    gm = GoDecMSE(X, w.labels, w.ranks, w.K, seed=w.seed)
    gm.step(10)
    Ls, S, idx, val = gpu_state(gm)
    ref = M.mse_train(w.X, w.labels, w.ranks, w.K, w.seed, 10)
    for i in range(len(w.labels)):
        assert rel(Ls[i], ref.Ls[i]) < 1e-10
        # the bases C^i agree through their projectors (reading M7)
        _, V = gm.factors(i)
        V = V.double().cpu().numpy()
        B = M.basis(ref.Ls[i])
        assert rel(V @ V.T, B @ B.T) < 1e-10
    assert rel(S, ref.S) < 1e-10
    info = gm.info()
    assert abs(info["rel_err_sq"] - ref.rel_err_sq[-1]) / ref.rel_err_sq[-1] < 1e-10
    gm.close()


def edge_workload(seed=21):
    """Labels: one empty, one with 3 rows and rank 5, overlapping others; two
    samples carry no label; K = 2 % of the entries."""
    rng = np.random.default_rng(seed)
    n, p = 300, 70
    X = rng.standard_normal((n, p))
    labels = [np.sort(rng.choice(n, 120, replace=False)), np.array([], np.int64),
              np.array([5, 77, 200]), np.sort(rng.choice(n, 90, replace=False))]
    # samples 10 and 11 carry no label
    labels = [np.setdiff1d(L, [10, 11]).astype(np.int64) for L in labels]
    w = wl.MseWorkload("edge", X, labels, [3, 2, 5, 4], int(0.02 * n * p), 3, seed)
    return w


def test_per_step_edge_cases_fp64():
    per_step(edge_workload(), np.float64, 3, 1e-10, "edge")


def test_per_step_k0_fp64():
    w = edge_workload(22)
    w.K = 0
    per_step(w, np.float64, 2, 1e-10, "K=0")


def test_disjoint_labels_recovered_in_one_sweep():
    from paper_1309_0302_amd.binding import GoDecMSE
    rng = np.random.default_rng(23)
    n, p, k = 500, 60, 5
    owner = rng.integers(0, k, size=n)
    ranks = [2, 3, 1, 4, 2]
    X = np.zeros((n, p))
    labels, parts = [], []
    for i in range(k):
        rows = np.flatnonzero(owner == i).astype(np.int64)
        P = rng.standard_normal((rows.size, ranks[i])) @ rng.standard_normal((ranks[i], p))
        X[rows] = P
        labels.append(rows)
        parts.append(P)
    gm = GoDecMSE(torch.from_numpy(X).cuda(), labels, ranks, 0, seed=3)
    gm.step(1)
    Ls, _, _, _ = gpu_state(gm)
    for L, P in zip(Ls, parts):
        assert rel(L, P) < 1e-12
    assert gm.info()["rel_err_sq"] < 1e-24
    gm.close()


def test_run_to_run_bit_identity_fp32():
    from paper_1309_0302_amd.binding import GoDecMSE
    w = wl.mse1(dtype=np.float32)
    X = torch.from_numpy(w.X).cuda()
    outs = []
    for _ in range(2):
        gm = GoDecMSE(X, w.labels, w.ranks, w.K, seed=w.seed)
        gm.step(3)
        U, V = gm.factors(3)
        idx, val = gm.S()
        info = gm.info()
        outs.append((U.cpu().numpy().copy(), V.cpu().numpy().copy(), idx.cpu().numpy().copy(),
                     val.cpu().numpy().copy(), np.float64(info["rel_err_sq"])))
        gm.close()
    for x, y in zip(*outs):
        assert np.array_equal(np.atleast_1d(x).view(np.uint8), np.atleast_1d(y).view(np.uint8))


def test_full_size_mse2_fp32_two_steps():
    per_step(wl.mse2(), np.float32, 2, 1e-5, "mse2")
