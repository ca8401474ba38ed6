"""HBM traffic of one GoDec iteration from rocprofv3 byte counters.

Two modes, run from the repository root:

    python -m paper_1309_0302_amd.profiling solve --form bf16_refine --steps 30
        one solve of the 10000 x 10000, rank 20 workload with the settings
        bench.py times (seed 1003, q = 2, one FP32 refinement iteration for
        the bf16_refine form), and nothing else; run it under
        `rocprofv3 --pmc FETCH_SIZE` and again under `--pmc WRITE_SIZE`
    python -m paper_1309_0302_amd.profiling copy
        a plain 1 GiB device-to-device copy, the calibration of the counters
    python -m paper_1309_0302_amd.profiling record --form bf16_refine \\
            --steps 30 FETCH.csv WRITE.csv COPY_FETCH.csv COPY_WRITE.csv
        prints the JSON line bench.py reads: the counters of every dispatch
        of the solve's iterations (from the first kernel of iteration 0 to
        the end), each counter scaled by (copy bytes) / (what it read for the
        copy), divided by the number of iterations, with the SHA-256 of every
        library source so that a changed kernel invalidates the record.

FETCH_SIZE and WRITE_SIZE are reported in KiB per dispatch.
"""
import argparse
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
COPY_BYTES = 1 << 30
FIRST_ITERATION_KERNEL = "k_copy_panel"   # the first kernel of every iteration


def source_hashes():
    out = {}
    for sub in ("paper_1309_0302_amd/csrc", "include"):
        d = os.path.join(ROOT, sub)
        for f in sorted(os.listdir(d)):
            if f.endswith((".hip", ".h")):
                p = os.path.join(d, f)
                out[f"{sub}/{f}"] = hashlib.sha256(open(p, "rb").read()).hexdigest()
    return out


def read_dispatches(path, counter):
    """(dispatch id, kernel name, value) of `counter`, in dispatch order."""
    rows = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            d = int(r["Dispatch_Id"])
            rows[d] = (r["Kernel_Name"], rows.get(d, ("", 0.0))[1] + float(r["Counter_Value"]))
    return [(d, *rows[d]) for d in sorted(rows)]


def solve_kib(path, counter):
    disp = read_dispatches(path, counter)
    start = next(i for i, (_, name, _) in enumerate(disp) if FIRST_ITERATION_KERNEL in name)
    return sum(v for _, _, v in disp[start:]), len(disp) - start


def copy_kib(path, counter):
    disp = read_dispatches(path, counter)
    vals = [v for _, name, v in disp if "copy" in name.lower() or "elementwise" in name.lower()]
    if not vals:
        raise SystemExit(f"no copy dispatch with {counter} in {path}")
    vals.sort()
    return vals[len(vals) // 2]


def cmd_solve(args):
    import torch
    from paper_1309_0302_amd import binding, workloads
    w = workloads.w3(seed=args.seed)
    X = torch.from_numpy(w.X).cuda()
    prec = binding.GODEC_PREC_BF16_REFINE if args.form == "bf16_refine" else \
        binding.GODEC_PREC_NATIVE
    g = binding.GoDec(X, w.r, w.k, w.q, seed=args.seed, prec=prec, refine_iters=1)
    torch.cuda.synchronize()
    g.step(args.steps, args.steps)
    torch.cuda.synchronize()
    g.close()
    print(f"[profiling] solve {args.form} {args.steps} iterations done", flush=True)


def cmd_copy(args):
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("[profiling] copy done", flush=True)


def cmd_record(args):
    f_kib, nd = solve_kib(args.fetch, "FETCH_SIZE")
    w_kib, _ = solve_kib(args.write, "WRITE_SIZE")
    cf = COPY_BYTES / (copy_kib(args.copy_fetch, "FETCH_SIZE") * 1024.0)
    cw = COPY_BYTES / (copy_kib(args.copy_write, "WRITE_SIZE") * 1024.0)
    fetch = f_kib * 1024.0 * cf / args.steps
    write = w_kib * 1024.0 * cw / args.steps
    rec = {"form": args.form, "steps": args.steps, "dispatches": nd,
           "fetch_bytes_per_iteration": round(fetch), "write_bytes_per_iteration": round(write),
           "hbm_bytes_per_iteration": round(fetch + write),
           "copy_scale_fetch": round(cf, 4), "copy_scale_write": round(cw, 4),
           "sources": source_hashes()}
    print(json.dumps(rec))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("solve")
    s.add_argument("--form", choices=["bf16_refine", "fp32"], default="bf16_refine")
    s.add_argument("--steps", type=int, default=30)
    s.add_argument("--seed", type=int, default=1003)
    sub.add_parser("copy")
    r = sub.add_parser("record")
    r.add_argument("--form", choices=["bf16_refine", "fp32"], default="bf16_refine")
    r.add_argument("--steps", type=int, default=30)
    r.add_argument("fetch")
    r.add_argument("write")
    r.add_argument("copy_fetch")
    r.add_argument("copy_write")
    args = ap.parse_args(argv)
    {"solve": cmd_solve, "copy": cmd_copy, "record": cmd_record}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
