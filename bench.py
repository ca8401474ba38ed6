"""Benchmark of GoDec by bilateral random projection on one MI355X.

    python bench.py [--gpus 1] [--steps 30] [--warmup 5]

Workload: the 10000 x 10000 FP32 matrix X = U V^T + S0 + G (U, V 10000 x 20,
unit-variance U V^T entries; 2e6 sparse entries U[-5, 5]; noise std 0.01),
r = 20, k = 2e6, q = 2, synthetic and seeded (paper_1309_0302_amd.workloads).
A step is one GoDec iteration (Algorithm 1: the BRP low-rank update with the
power scheme, then the top-k sparse update) over the whole matrix, with X
already resident in device memory.  `--steps K` iterations are timed as one
solve from S_0 = 0; in the headline mixed-precision form the last iteration
is the FP32 refinement.  The same K iterations are also timed in plain FP32.

Prints one JSON line with:
- the headline value (iterations/s of the bf16 + refinement form) and the
  FP32 plain figure beside it;
- `roofline`: the per-iteration fraction of the HBM roofline, i.e. the
  algorithmic bytes of one iteration (one read of D per panel pass, one read
  of X for the residual and selection, the S corrections and the S write;
  `iteration_bytes`) over the measured time per iteration, against 8 TB/s;
  the dominant kernel's own figure (its launches stamped with their start
  and end on the library's stream) is reported inside it;
- `precision_vs_oracle`: the relative errors of L, S and the objective of
  both forms after K iterations against the FP64 oracle's own K-iteration run
  on the same X and A1 (common-support S error and boundary swaps counted
  separately);
- `cpu_baseline`: the FP64 oracle on the host cores, on the same workload
  (its per-iteration median) and on the 500 x 500 FP64 and 25344 x 200 FP32
  workloads, with all threads and with one;
- GPU legs on those two small workloads, and the secondary forms (batched,
  differentiable layer, projection form, warm start, completion, GreBsmo).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("GoDec-BRP iter/s @10k×10k r=20: BF16-MFMA+refine vs FP32 plain "
          "at 1e-5 err")
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def rel_diff_factors(a_l, a_r, b_l, b_r):
    """||A_l A_r^T - B_l B_r^T||_F / ||B_l B_r^T||_F in FP64 on the device."""
    import torch

    def inner(p1, q1, p2, q2):
        return float(torch.sum((p1.T @ p2) * (q1.T @ q2)))
    a_l, a_r, b_l, b_r = (t.double() for t in (a_l, a_r, b_l, b_r))
    aa = inner(a_l, a_r, a_l, a_r)
    bb = inner(b_l, b_r, b_l, b_r)
    ab = inner(a_l, a_r, b_l, b_r)
    return max(aa - 2 * ab + bb, 0.0) ** 0.5 / bb ** 0.5


def run_form(X, w, prec, steps, warmup, seed, lstep=0, warm_start=0, q=None, redraw_a1=0):
    """Time `steps` iterations (one solve); returns timing, stats, factors.
    lstep = 1 takes the projection form of the L update; warm_start = 1
    starts each power chain from the previous Q2; redraw_a1 = 1 draws a new
    A1 every iteration; q overrides w.q."""
    q = w.q if q is None else q
    import torch
    from paper_1309_0302_amd.binding import GoDec
    stream = torch.cuda.current_stream()
    if warmup > 0:
        g = GoDec(X, w.r, w.k, q, seed=seed, prec=prec, refine_iters=1, lstep=lstep,
                  warm_start=warm_start, redraw_a1=redraw_a1)
        g.step(warmup, warmup)
        g.info()
        g.close()
    g = GoDec(X, w.r, w.k, q, seed=seed, prec=prec, refine_iters=1, lstep=lstep,
              warm_start=warm_start, redraw_a1=redraw_a1)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    g.step(steps, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    info = g.info()
    UL, VL = g.factors()
    s_idx, s_val = g.S()
    g.close()
    # the same solve again with per-kernel event timing switched on
    g = GoDec(X, w.r, w.k, q, seed=seed, prec=prec, refine_iters=1, lstep=lstep,
              warm_start=warm_start, redraw_a1=redraw_a1)
    g.profile(True)
    g.step(steps, steps)
    stats = g.profile_read()
    g.profile(False)
    g.close()
    return dict(ms=ev_ms, wall_s=wall, info=info, UL=UL, VL=VL, s_idx=s_idx, s_val=s_val,
                stats=stats)


COUNTERS_FILE = os.path.join(ROOT, "profiles", "godec_w3_iteration_hbm_counters.md")


def measured_traffic(mixed):
    """HBM bytes per iteration of the timed form from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE record (each scaled by what the counter
    reads for a plain copy of known size), or None when there is no record
    for this form or any kernel source has changed since the counters were
    taken (the record carries the SHA-256 of every source file)."""
    import hashlib
    if not os.path.exists(COUNTERS_FILE):
        return None
    recs = []
    for line in open(COUNTERS_FILE):
        line = line.strip()
        if line.startswith("{") and '"hbm_bytes_per_iteration"' in line:
            recs.append(json.loads(line))
    want = "bf16_refine" if mixed else "fp32"
    rec = next((r for r in recs if r.get("form") == want), None)
    if rec is None:
        return None
    for path, sha in rec.get("sources", {}).items():
        src = os.path.join(ROOT, path)
        if not os.path.exists(src) or \
                hashlib.sha256(open(src, "rb").read()).hexdigest() != sha:
            return None
    return rec["hbm_bytes_per_iteration"]


def iteration_bytes(m, n, k, q, panel_elem, res_elem=4, refine=False):
    """Algorithmic HBM bytes of one GoDec iteration of the restated
    Algorithm 1 (Sec. 3.1.3): 3q + 2 panel passes that each stream D = X - S
    once (2q + 1 Gram passes of the subspace chain, q of the B chain and the
    plain B' = D Y pass), one residual / selection read of X, 8 bytes of S
    correction per entry of S for every panel pass, and 20 bytes per entry
    of S for the S write and the selection candidates.  In the refinement
    iteration of the mixed form the last subspace pass and the whole B chain
    read FP32 (4-byte) D instead of the bf16 copy."""
    mn = m * n
    passes = 3 * q + 2
    if refine:
        panel = (2 * q) * 2 * mn + (q + 2) * 4 * mn
    else:
        panel = passes * panel_elem * mn
    return panel + res_elem * mn + passes * 8 * k + 20 * k


def roofline_of(stats, m, n, k, q, steps, ms, mixed, refine_iters=1, elem=4):
    """Per-iteration HBM roofline fraction of a timed solve of `steps`
    iterations taking `ms`: the average algorithmic bytes of its iterations
    over the measured time per iteration, against the 8 TB/s peak.  The
    dominant kernel's own bandwidth is reported inside."""
    if mixed:
        nref = min(refine_iters, steps)
        b_avg = ((steps - nref) * iteration_bytes(m, n, k, q, 2)
                 + nref * iteration_bytes(m, n, k, q, 2, refine=True)) / steps
    else:
        b_avg = iteration_bytes(m, n, k, q, elem, res_elem=elem)
    t_iter = ms / steps * 1e-3
    achieved = b_avg / t_iter / 1e9
    dom = max(stats, key=lambda st: st["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    dom_gbs = dom["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
    streamed = sum(st["bytes_per_launch"] * st["launches"] for st in stats) / steps
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(mixed),
            "algorithmic_bytes_per_iteration": round(b_avg),
            "ms_per_iteration": round(ms / steps, 4),
            "streamed_bytes_per_iteration": round(streamed),
            "streamed_over_algorithmic": round(streamed / b_avg, 3),
            "dominant_kernel": {"name": dom["name"], "launches": dom["launches"],
                                "avg_launch_us": round(avg_ms * 1e3, 2),
                                "algorithmic_bytes_per_launch": dom["bytes_per_launch"],
                                "achieved_GBps": round(dom_gbs, 1),
                                "frac": round(dom_gbs / HBM_PEAK_GBS, 4)}}


def trajectory_errors(X, UL, VL, s_idx, s_val, thr, L_o, S_o, thr_o):
    """Errors of a GPU run (factors UL, VL; S as sorted linear indices and
    values; threshold thr) against the oracle's own run (dense L_o, S_o and
    its threshold) on the same X, all in FP64 on the host:
    rel_L = ||L - L_o||_F / ||L_o||_F; rel_obj = |e - e_o| / e_o with
    e = ||X - L - S||_F^2 / ||X||_F^2 computed from the arrays; the S error on
    the common support and over everything; and the boundary swaps (entries
    in one support only).  A swap is within the band when its oracle
    residual lies within 2 max|L - L_o| + |thr - thr_o| of the oracle's
    threshold."""
    import numpy as np
    X = np.asarray(X, dtype=np.float64)
    L = np.asarray(UL, np.float64) @ np.asarray(VL, np.float64).T
    nl = np.linalg.norm(L_o)
    dL = L - L_o
    rel_L = float(np.linalg.norm(dL) / nl)
    band_L = float(np.max(np.abs(dL)))
    del dL
    idx = np.asarray(s_idx, np.int64)
    val = np.asarray(s_val, np.float64)
    Sf = S_o.ravel()
    idx_o = np.flatnonzero(Sf)
    common, ia, ib = np.intersect1d(idx, idx_o, assume_unique=True, return_indices=True)
    vo = Sf[idx_o]
    rel_S_common = float(np.linalg.norm(val[ia] - vo[ib]) / max(np.linalg.norm(vo[ib]), 1e-300))
    only_g = np.setdiff1d(idx, idx_o, assume_unique=True)
    only_o = np.setdiff1d(idx_o, idx, assume_unique=True)
    # ||S - S_o||^2 over the union: common part plus each side's own entries
    ga = np.ones(idx.size, bool)
    ga[ia] = False
    ob = np.ones(idx_o.size, bool)
    ob[ib] = False
    d2 = (np.sum((val[ia] - vo[ib]) ** 2) + np.sum(val[ga] ** 2) + np.sum(vo[ob] ** 2))
    rel_S = float(np.sqrt(d2) / max(np.linalg.norm(vo), 1e-300))
    xx = float(np.sum(X * X))
    E = X - L
    Ef = E.ravel()
    Ef[idx] -= val
    e = float(np.sum(E * E)) / xx
    del E, Ef
    E_o = X - L_o - S_o
    e_o = float(np.sum(E_o * E_o)) / xx
    del E_o
    swaps = np.concatenate([only_g, only_o])
    Xf = X.ravel()
    band = 2.0 * band_L + abs(thr - thr_o)
    if swaps.size:
        r_o = np.abs(Xf[swaps] - L_o.ravel()[swaps])
        dist = np.abs(r_o - thr_o)
        worst = float(np.max(dist))
    else:
        worst = 0.0
    return {"rel_L": rel_L, "rel_obj": abs(e - e_o) / e_o if e_o > 0 else abs(e - e_o),
            "obj": e, "obj_oracle": e_o,
            "rel_S_common": rel_S_common, "rel_S": rel_S,
            "common": int(common.size), "swaps": int(swaps.size),
            "swaps_gpu_only": int(only_g.size), "swaps_oracle_only": int(only_o.size),
            "swap_band": band, "swap_worst_dist": worst,
            "swaps_within_band": bool(worst <= band), "max_abs_dL": band_L}


def run_batched(iters, warmup, seed=1004):
    """The 64-problem workload (uneven shapes, q = 1) in the batched form:
    `iters` graph-replayed iterations from S_0 = 0, timed on the batch's
    stream with HIP events."""
    import numpy as np
    import torch
    from paper_1309_0302_amd import workloads
    from paper_1309_0302_amd.binding import GoDecBatch
    works = workloads.w4(seed=seed)
    specs = [(torch.from_numpy(w.X).cuda(), w.r, w.k, 100 + i) for i, w in enumerate(works)]
    torch.cuda.synchronize()
    if warmup > 0:
        gb = GoDecBatch(specs, 1)
        gb.step(warmup)
        gb.synchronize()
        gb.close()
    gb = GoDecBatch(specs, 1)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    gb.synchronize()
    e0.record(gb.stream)
    gb.step(iters)
    e1.record(gb.stream)
    gb.synchronize()
    ms = e0.elapsed_time(e1)
    rows, items = gb.tuning()
    mn = sum(int(w.X.shape[0]) * int(w.X.shape[1]) for w in works)
    # algorithmic bytes of one batch iteration: 2q+1 + q Gram passes, the
    # B' pass and two selection passes, each reading every X or D once
    passes = (2 * 1 + 1) + 1 + 1 + 2
    bytes_iter = passes * mn * 4
    rel = [gb.info(i)["rel_err_sq"] for i in range(len(works))]
    gb.close()
    ms_iter = ms / iters
    achieved = bytes_iter / (ms_iter * 1e-3) / 1e9
    return {"workload": f"w4_{len(works)}_problems_q1", "problems": len(works),
            "sum_mn": mn, "iterations": iters,
            "ms_per_iteration": round(ms_iter, 4),
            "problem_iterations_per_s": round(len(works) * iters / (ms * 1e-3), 1),
            "rows_per_item": rows, "work_items": items,
            "algorithmic_bytes_per_iteration": bytes_iter,
            "achieved_GBps": round(achieved, 1),
            "frac_of_hbm_peak": round(achieved / HBM_PEAK_GBS, 4),
            "median_final_rel_err_sq": float(np.median(rel))}


def run_layer(warmup, seed=1005):
    """The differentiable layer on its 16 x 4096 x 256 FP32 workload (r = 4,
    k = 5 %, q = 1, T = 10): forward, then the hand-written backward of the
    loss ||S - S_tgt||^2 + ||L - L_tgt||^2, each timed on the host around a
    synchronised call."""
    import torch
    from paper_1309_0302_amd import workloads
    from paper_1309_0302_amd.binding import GoDecLayer
    w = workloads.w5(seed=seed)
    X = torch.from_numpy(w["X"]).cuda()
    Lt = torch.from_numpy(w["L_target"]).cuda()
    St = torch.from_numpy(w["S_target"]).cuda()
    nb, m, n = X.shape
    fwd, bwd = [], []
    for it in range(warmup + 1):
        layer = GoDecLayer(w["r"], w["k"], w["q"], w["iters"], seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L, S = layer.forward(X)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dL = 2 * (L - Lt)
        dS = 2 * (S - St)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        dX = layer.backward(dL, dS)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        layer.close()
        fwd.append((t1 - t0) * 1e3)
        bwd.append((t3 - t2) * 1e3)
    assert bool(torch.isfinite(dX).all())
    p, q, T = 2 * w["q"] + 1, w["q"], w["iters"]
    # algorithmic bytes of the backward: per unrolled step the forward panels
    # of f read D p + q + 1 times (each A P = D^T (D P) in one read), the
    # adjoint reads L^bar twice and D 1 + q + p times (each pair of rank terms
    # together with the next power of A in one read); D = X - S reads X and
    # writes D; X^bar is read and written and L^bar written once
    reads = (p + q + 1) + 2 + (1 + q + p)
    bytes_bwd = T * (reads + 2 + 3) * nb * m * n * 4
    return {"workload": f"w5_{nb}x{m}x{n}_r{w['r']}_T{T}_f32", "batch": nb,
            "forward_ms": round(fwd[-1], 3), "backward_ms": round(bwd[-1], 3),
            "fwd_bwd_ms": round(fwd[-1] + bwd[-1], 3),
            "backward_algorithmic_bytes": bytes_bwd,
            "backward_achieved_GBps": round(bytes_bwd / (bwd[-1] * 1e-3) / 1e9, 1)}


def grebsmo_bytes(m, n, r, dr, K, power, elem=4):
    """Algorithmic bytes of one GreBsmo solve: per stage the greedy step's
    power Gram passes (two reads of R each), one read of D for the stage's
    first D V^T, and per inner iteration the transposed pass (read D) and the
    soft pass (read X, write D; it also forms the next D V^T), plus the R
    write of every stage but the last."""
    stages = -(-r // dr)
    mn = m * n * elem
    return stages * (2 * power + 1 + 3 * K) * mn + (stages - 1) * mn


def run_grebsmo(warmup, seed=1007):
    """GreBsmo on the 25 344 x 500 FP32 video-shaped workload (r = 4, dr = 1,
    K = 10, lambda = 0.125, power = 2): whole solves, timed on the stream with
    HIP events; the FP64 oracle's solve on the host beside it."""
    import numpy as np
    import torch
    from paper_1309_0302_amd import workloads
    from paper_1309_0302_amd.binding import GreBsmo
    w = workloads.g2(seed=seed)
    X = torch.from_numpy(w.X).cuda()
    m, n = w.X.shape
    ms = []
    for it in range(warmup + 3):
        gb = GreBsmo(X, w.r, dr=w.dr, power=w.power, lam=w.lam, seed=w.seed)
        stream = torch.cuda.ExternalStream(gb.stream) if gb.stream else \
            torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        gb.solve(w.K, 0.0, want_info=False)
        e1.record(stream)
        torch.cuda.synchronize()
        if it >= warmup:
            ms.append(e0.elapsed_time(e1))
        info = gb.info()
        gb.close()
    t = float(np.median(ms))
    nbytes = grebsmo_bytes(m, n, w.r, w.dr, w.K, w.power)
    return {"workload": w.name, "m": m, "n": n, "r": w.r, "dr": w.dr, "K": w.K,
            "lambda": w.lam, "power": w.power, "ms_per_solve": round(t, 4),
            "solves_per_s": round(1e3 / t, 2),
            "inner_iterations": int(info.inner_iters),
            "algorithmic_bytes_per_solve": nbytes,
            "achieved_GBps": round(nbytes / (t * 1e-3) / 1e9, 1),
            "frac_of_hbm_peak": round(nbytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "rel_err_sq": info.rel_err_sq, "nnz": int(info.nnz)}


def grebsmo_cpu_baseline(seed=1007):
    """The FP64 GreBsmo oracle on the host cores: one whole solve of the same
    workload."""
    import numpy as np
    from oracle import grebsmo_ref as g
    from oracle.rng_ref import a1_gaussian
    from paper_1309_0302_amd import workloads
    try:
        from threadpoolctl import threadpool_info
        threads = max(i.get("num_threads", 1) for i in threadpool_info()) or 1
    except Exception:
        threads = os.cpu_count() or 1
    w = workloads.g2(seed=seed)
    Om = a1_gaussian(w.seed, w.X.shape[1], w.r)
    X = w.X.astype(np.float64)
    t0 = time.perf_counter()
    g.grebsmo(X, w.r, w.dr, w.K, w.lam, w.power, Om)
    dt = time.perf_counter() - t0
    return {"value": round(1.0 / dt, 4), "unit": "solves/s", "cores": threads,
            "kind": "oracle",
            "sample": f"one FP64 oracle solve of the full {w.X.shape[0]}x{w.X.shape[1]} "
                      f"GreBsmo workload (numpy/OpenBLAS), {dt:.1f} s"}


def run_completion(X, w, iters, warmup, frac=0.1, seed=1008):
    """Matrix completion (fixed support) on the 10 000 x 10 000 FP32 matrix
    with a seeded 10 % of its entries unobserved: `iters` iterations from
    S_0 = 0, timed on the stream with HIP events."""
    import numpy as np
    import torch
    from paper_1309_0302_amd import workloads
    from paper_1309_0302_amd.binding import GoDec
    m, n = X.shape
    sup = torch.from_numpy(workloads.missing_support(m, n, frac, seed)).cuda()
    gd = GoDec(X, w.r, int(sup.numel()), w.q, seed=w.seed, support=sup)
    gd.step(warmup)
    torch.cuda.synchronize()
    gd.close()
    gd = GoDec(X, w.r, int(sup.numel()), w.q, seed=w.seed, support=sup)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    gd.step(iters)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    info = gd.info()
    UL, VL = gd.factors()
    gd.close()
    out = {"workload": f"m1_{m}x{n}_r{w.r}_q{w.q}_missing{frac:g}_f32",
           "unobserved": int(sup.numel()), "iterations": iters,
           "ms_per_iteration": round(ms / iters, 4),
           "iter_per_s": round(iters * 1e3 / ms, 2),
           "rel_err_sq_observed": info["rel_err_sq"]}
    # the BF16 panel form (last iteration refined in FP32), same solve
    from paper_1309_0302_amd.binding import GODEC_PREC_BF16_REFINE
    gb = GoDec(X, w.r, int(sup.numel()), w.q, seed=w.seed, support=sup,
               prec=GODEC_PREC_BF16_REFINE)
    torch.cuda.synchronize()
    e0.record()
    gb.step(iters, iters)
    e1.record()
    torch.cuda.synchronize()
    msb = e0.elapsed_time(e1)
    infob = gb.info()
    ULb, VLb = gb.factors()
    gb.close()
    out["bf16_refine"] = {"ms_per_iteration": round(msb / iters, 4),
                          "iter_per_s": round(iters * 1e3 / msb, 2),
                          "rel_err_sq_observed": infob["rel_err_sq"],
                          "rel_diff_L_vs_f32": rel_diff_factors(ULb, VLb, UL, VL)}
    return out


def mse_bytes(w):
    """Algorithmic bytes of one MSE training iteration (Algorithm 4): per
    label two reads of its rows of the residual (N A1 with N^T Y1 in one
    read, then N Y2) and one write of them, the sparse step's read of
    X - sum L, 20 bytes per entry of S for the S write and candidates, and
    two scattered S updates of the residual (12 bytes each per entry)."""
    n, p = w.X.shape
    rows = sum(len(r) for r in w.labels)
    return 3 * rows * p * 4 + n * p * 4 + 20 * w.K + 24 * w.K


def run_mse(warmup, iters=10, skip_cpu=False):
    """MSE training on the 65 536 x 512 FP32 multi-label workload (32 labels,
    ranks 2..8, K = 2 % of the entries): `iters` iterations timed on the
    stream with HIP events; the FP64 oracle's first iteration on the host."""
    import numpy as np
    import torch
    from paper_1309_0302_amd import workloads
    from paper_1309_0302_amd.binding import GoDecMSE
    w = workloads.mse2()
    X = torch.from_numpy(w.X).cuda()
    stream = torch.cuda.current_stream()
    ms = []
    for it in range(warmup + 3):
        gm = GoDecMSE(X, w.labels, w.ranks, w.K, seed=w.seed)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        gm.step(iters)
        e1.record(stream)
        torch.cuda.synchronize()
        if it >= warmup:
            ms.append(e0.elapsed_time(e1))
        info = gm.info()
        gm.close()
    t = float(np.median(ms)) / iters
    nb = mse_bytes(w)
    out = {"workload": w.name, "n": int(w.X.shape[0]), "p": int(w.X.shape[1]),
           "labels": len(w.labels), "label_rows": int(sum(len(r) for r in w.labels)),
           "K": w.K, "iterations": iters, "ms_per_iteration": round(t, 4),
           "iter_per_s": round(1e3 / t, 2), "algorithmic_bytes_per_iteration": nb,
           "achieved_GBps": round(nb / (t * 1e-3) / 1e9, 1),
           "frac_of_hbm_peak": round(nb / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "rel_err_sq": info["rel_err_sq"]}
    if not skip_cpu:
        from oracle import mse_ref as M
        bl = blas_info()
        tr = M.mse_train(w.X.astype(np.float64), w.labels, w.ranks, w.K, w.seed, 1)
        out["cpu_baseline"] = {"value": round(1.0 / tr.seconds[0], 4), "unit": "iter/s",
                               "cores": bl["threads"] or os.cpu_count(), "kind": "oracle",
                               "sample": f"one FP64 oracle iteration of the full workload "
                                         f"({tr.seconds[0]:.1f} s)"}
    return out


def run_copy(nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of a known size: the reference against
    which the HBM byte counters of the other kernels are scaled."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return {"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps,
            "ms_per_copy": round(dt * 1e3, 4),
            "GBps_read_plus_write": round(2 * nbytes / dt / 1e9, 1)}


def blas_info():
    """BLAS library and thread count numpy uses (threadpoolctl)."""
    try:
        from threadpoolctl import threadpool_info
        infos = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if infos:
            i = infos[0]
            return {"vendor": i.get("internal_api"), "threads": i.get("num_threads"),
                    "version": i.get("version")}
    except Exception:
        pass
    return {"vendor": None, "threads": None, "version": None}


def oracle_run(w, iters, threads=None):
    """The FP64 oracle's own `iters`-iteration run of workload w (A1 from the
    workload's seed), on `threads` BLAS threads (None: all)."""
    import numpy as np
    from oracle import godec_ref as g
    from oracle.rng_ref import a1_gaussian
    A1 = a1_gaussian(w.seed, w.X.shape[1], w.r)
    X = w.X.astype(np.float64)
    if threads is None:
        return g.godec_brp(X, w.r, w.k, w.q, A1, iters)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=threads, user_api="blas"):
        return g.godec_brp(X, w.r, w.k, w.q, A1, iters)


def oracle_rate(tr):
    import numpy as np
    med = float(np.median(tr.seconds))
    return {"iter_per_s": round(1.0 / med, 4), "median_s_per_iter": round(med, 5),
            "iters": len(tr.seconds), "total_s": round(float(np.sum(tr.seconds)), 3)}


def run_small_leg(w, prec, reps=5):
    """GPU leg on a small workload (its own T iterations per solve, FP64 or
    FP32 native): the median over `reps` timed solves, each timed on the
    stream with HIP events; returns the rate and the last solve's results."""
    import numpy as np
    import torch
    from paper_1309_0302_amd.binding import GoDec
    X = torch.from_numpy(w.X).cuda()
    stream = torch.cuda.current_stream()
    ms = []
    for it in range(reps + 1):
        g = GoDec(X, w.r, w.k, w.q, seed=w.seed, prec=prec)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.step(w.iters, w.iters)
        e1.record(stream)
        torch.cuda.synchronize()
        if it > 0:
            ms.append(e0.elapsed_time(e1))
        if it < reps:
            g.close()
    info = g.info()
    UL, VL = g.factors()
    idx, val = g.S()
    out = dict(UL=UL.double().cpu().numpy(), VL=VL.double().cpu().numpy(),
               idx=idx.cpu().numpy(), val=val.double().cpu().numpy(), info=info)
    g.close()
    t = float(np.median(ms))
    return t, out


def host_errors(X, form, tr):
    """trajectory_errors of a timed GPU form against the oracle's run."""
    return trajectory_errors(X, form["UL"].double().cpu().numpy(),
                             form["VL"].double().cpu().numpy(),
                             form["s_idx"].cpu().numpy(), form["s_val"].double().cpu().numpy(),
                             form["info"]["threshold"], tr.L, tr.S, tr.thresholds[-1])


def small_legs(skip_cpu):
    """GPU legs on the 500 x 500 FP64 (T = 20) and 25 344 x 200 FP32 (T = 50)
    workloads, each against the oracle's own run (all host threads), with the
    oracle's rate on all threads and on one."""
    from paper_1309_0302_amd import workloads
    from paper_1309_0302_amd.binding import GODEC_PREC_NATIVE
    legs = {}
    for w in (workloads.w1(), workloads.w2()):
        m, n = w.X.shape
        name = w.name
        log(f"[bench] small leg {name}: {w.iters} iterations")
        t, res = run_small_leg(w, GODEC_PREC_NATIVE)
        leg = {"m": m, "n": n, "r": w.r, "k": w.k, "q": w.q, "iterations_per_solve": w.iters,
               "ms_per_solve": round(t, 4), "iter_per_s": round(w.iters / (t * 1e-3), 1),
               "algorithmic_bytes_per_iteration": iteration_bytes(
                   m, n, w.k, w.q, w.X.dtype.itemsize, res_elem=w.X.dtype.itemsize)}
        if not skip_cpu:
            tr = oracle_run(w, w.iters)
            leg["vs_oracle"] = trajectory_errors(w.X, res["UL"], res["VL"], res["idx"],
                                                 res["val"], res["info"]["threshold"],
                                                 tr.L, tr.S, tr.thresholds[-1])
            tr1 = oracle_run(w, w.iters, threads=1)
            leg["cpu_baseline"] = {"all_threads": oracle_rate(tr), "one_thread": oracle_rate(tr1)}
        legs[name] = leg
    return legs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=1003)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-fp32", action="store_true")
    ap.add_argument("--skip-small", action="store_true")
    ap.add_argument("--skip-batch", action="store_true")
    ap.add_argument("--batch-iters", type=int, default=25)
    ap.add_argument("--skip-layer", action="store_true")
    ap.add_argument("--skip-copy", action="store_true")
    ap.add_argument("--skip-grebsmo", action="store_true")
    ap.add_argument("--skip-completion", action="store_true")
    ap.add_argument("--skip-projection", action="store_true")
    ap.add_argument("--skip-warm", action="store_true")
    ap.add_argument("--skip-redraw", action="store_true")
    ap.add_argument("--skip-mse", action="store_true")
    ap.add_argument("--only", choices=["batch", "layer", "copy", "grebsmo", "completion",
                                       "small", "mse"],
                    help="run one secondary leg alone (for profiling) and print its JSON")
    ap.add_argument("--size", type=int, default=10000,
                    help="square size (default: the 10000 x 10000 workload)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not "
              "supported (the row-block sharding across GPUs is designed, not built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1309_0302_amd import workloads
    from paper_1309_0302_amd.binding import GODEC_PREC_BF16_REFINE, GODEC_PREC_NATIVE

    if args.only == "batch":
        print(json.dumps(run_batched(args.batch_iters, min(args.warmup, 3))), flush=True)
        return
    if args.only == "layer":
        print(json.dumps(run_layer(min(args.warmup, 1))), flush=True)
        return
    if args.only == "copy":
        print(json.dumps(run_copy()), flush=True)
        return
    if args.only == "mse":
        print(json.dumps(run_mse(min(args.warmup, 2), skip_cpu=args.skip_cpu)), flush=True)
        return
    if args.only == "small":
        print(json.dumps(small_legs(args.skip_cpu)), flush=True)
        return
    if args.only == "grebsmo":
        out = run_grebsmo(min(args.warmup, 2))
        if not args.skip_cpu:
            out["cpu_baseline"] = grebsmo_cpu_baseline()
        print(json.dumps(out), flush=True)
        return

    log(f"[bench] generating workload {args.size}x{args.size}")
    w = workloads.w3(seed=args.seed, m=args.size, n=args.size)
    X = torch.from_numpy(w.X).cuda()
    torch.cuda.synchronize()
    m, n = w.X.shape
    if args.only == "completion":
        print(json.dumps(run_completion(X, w, 10, 2)), flush=True)
        return
    log("[bench] bf16 + refinement form")
    bf = run_form(X, w, GODEC_PREC_BF16_REFINE, args.steps, args.warmup, args.seed)
    log(f"[bench] bf16+refine {args.steps / (bf['ms'] * 1e-3):.1f} iter/s")
    fp = None
    if not args.skip_fp32:
        log("[bench] fp32 plain form")
        fp = run_form(X, w, GODEC_PREC_NATIVE, args.steps, args.warmup, args.seed)
        log(f"[bench] fp32 {args.steps / (fp['ms'] * 1e-3):.1f} iter/s")
    value = args.steps / (bf["ms"] * 1e-3)
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(bf["ms"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": w.name + "_f32", "m": m, "n": n, "r": w.r, "k": w.k, "q": w.q,
                   "iterations_per_solve": args.steps, "refine_iters": 1,
                   "form": "bf16 panels (fp32 accumulate) + fp32 refinement, "
                           "fp64 r x r core"},
        "roofline": roofline_of(bf["stats"], m, n, w.k, w.q, args.steps, bf["ms"], True),
        "final_rel_err_sq": bf["info"]["rel_err_sq"],
    }
    if fp is not None:
        out["fp32_plain"] = {"value": round(args.steps / (fp["ms"] * 1e-3), 2),
                             "ms_per_step": round(fp["ms"] / args.steps, 4),
                             "roofline": roofline_of(fp["stats"], m, n, w.k, w.q, args.steps,
                                                     fp["ms"], False),
                             "final_rel_err_sq": fp["info"]["rel_err_sq"]}
        out["speedup_vs_fp32_plain"] = round(value / out["fp32_plain"]["value"], 3)
        out["rel_diff_L_bf16_refine_vs_fp32"] = rel_diff_factors(
            bf["UL"], bf["VL"], fp["UL"], fp["VL"])
    out["kernels"] = bf["stats"]
    if not args.skip_copy:
        out["measured_copy"] = run_copy(1 << 30, 5)
    if not args.skip_small:
        out["small_workloads"] = small_legs(args.skip_cpu)
    if not args.skip_batch:
        log("[bench] batched form: 64 problems")
        out["batched"] = run_batched(args.batch_iters, min(args.warmup, 3))
        log(f"[bench] batched {out['batched']['ms_per_iteration']} ms/iteration")
    if not args.skip_layer:
        log("[bench] differentiable layer: 16 x 4096 x 256, T = 10")
        out["layer"] = run_layer(min(args.warmup, 1))
        log(f"[bench] layer fwd {out['layer']['forward_ms']} ms, "
            f"bwd {out['layer']['backward_ms']} ms")
    if not args.skip_projection:
        log("[bench] projection-form L update, bf16 + refinement")
        pj = run_form(X, w, GODEC_PREC_BF16_REFINE, args.steps, args.warmup, args.seed, lstep=1)
        out["projection_form"] = {
            "value": round(args.steps / (pj["ms"] * 1e-3), 2), "unit": "iter/s",
            "ms_per_step": round(pj["ms"] / args.steps, 4),
            "final_rel_err_sq": pj["info"]["rel_err_sq"],
            "rel_diff_L_vs_root_form": rel_diff_factors(pj["UL"], pj["VL"], bf["UL"], bf["VL"])}
        log(f"[bench] projection form {out['projection_form']['value']} iter/s")
    if not args.skip_warm:
        log("[bench] warm-started chains at q = 1, bf16 + refinement")
        wm = run_form(X, w, GODEC_PREC_BF16_REFINE, args.steps, args.warmup, args.seed,
                      warm_start=1, q=1)
        out["warm_start_q1"] = {
            "value": round(args.steps / (wm["ms"] * 1e-3), 2), "unit": "iter/s",
            "ms_per_step": round(wm["ms"] / args.steps, 4),
            "final_rel_err_sq": wm["info"]["rel_err_sq"],
            "rel_diff_L_vs_cold_q2": rel_diff_factors(wm["UL"], wm["VL"], bf["UL"], bf["VL"])}
        log(f"[bench] warm start q=1 {out['warm_start_q1']['value']} iter/s")
    if not args.skip_redraw:
        log("[bench] a new A1 every iteration, bf16 + refinement")
        rd = run_form(X, w, GODEC_PREC_BF16_REFINE, args.steps, args.warmup, args.seed,
                      redraw_a1=1)
        out["redraw_a1"] = {
            "value": round(args.steps / (rd["ms"] * 1e-3), 2), "unit": "iter/s",
            "ms_per_step": round(rd["ms"] / args.steps, 4),
            "final_rel_err_sq": rd["info"]["rel_err_sq"],
            "rel_diff_L_vs_fixed_a1": rel_diff_factors(rd["UL"], rd["VL"], bf["UL"], bf["VL"])}
        log(f"[bench] redraw_a1 {out['redraw_a1']['value']} iter/s")
    if not args.skip_completion:
        log("[bench] matrix completion: 10000 x 10000, 10 % unobserved")
        out["completion"] = run_completion(X, w, 10, 2)
        log(f"[bench] completion {out['completion']['iter_per_s']} iter/s")
    if not args.skip_mse:
        log("[bench] MSE training: 65536 x 512, 32 labels")
        out["mse"] = run_mse(min(args.warmup, 2), skip_cpu=args.skip_cpu)
        log(f"[bench] mse {out['mse']['ms_per_iteration']} ms/iteration")
    if not args.skip_grebsmo:
        log("[bench] GreBsmo: 25344 x 500 video-shaped, r = 4")
        out["grebsmo"] = run_grebsmo(min(args.warmup, 2))
        log(f"[bench] grebsmo {out['grebsmo']['ms_per_solve']} ms/solve")
    del X
    torch.cuda.empty_cache()
    if not args.skip_cpu:
        if "grebsmo" in out:
            log("[bench] grebsmo cpu baseline: one oracle solve")
            out["grebsmo"]["cpu_baseline"] = grebsmo_cpu_baseline()
        # the oracle's own run of the timed solve's iterations on the same X
        # and A1: the per-iteration CPU baseline, and the reference for the
        # errors of both GPU forms (skipped beyond 30 iterations, ~1 s each)
        iters = min(args.steps, 30)
        log(f"[bench] cpu baseline: {iters} oracle iterations of the full workload")
        tr = oracle_run(w, iters)
        rate = oracle_rate(tr)
        bl = blas_info()
        out["cpu_baseline"] = {
            "value": rate["iter_per_s"], "unit": "iter/s",
            "cores": bl["threads"] or os.cpu_count(), "kind": "oracle",
            "sample": f"{iters} FP64 oracle iterations of the full {m}x{n} workload "
                      f"(numpy/{bl['vendor']}, {bl['threads']} threads); value = 1 / median "
                      f"per-iteration time; {rate['total_s']} s",
            "host_cpu_count": os.cpu_count(), "blas": bl, "median_s_per_iter":
                rate["median_s_per_iter"]}
        if iters == args.steps:
            log("[bench] errors of both forms against the oracle's run")
            pv = {"iterations": iters, "bf16_refine": host_errors(w.X, bf, tr)}
            if fp is not None:
                pv["fp32_plain"] = host_errors(w.X, fp, tr)
            out["precision_vs_oracle"] = pv
        del tr
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
