#!/usr/bin/env python3
"""Throughput of the extra-component computation stage on one MI355X.

Workload: the Legendre transform of order N = 16384 (orthonormalised, Gauss-
Legendre nodes), 64 right-hand sides x ~ N(0, 1) (seed 1), eps1 = 1e-7,
eps2 = 1e-2, float64 precomputation.  One step = one spt_execute of all 64
right-hand sides (extend + window + FFT of every block, banded product of every
block and the direct tail).  The headline value is the split-bf16 path
(float32 FFT, bfloat16x3 matrix-core product accumulated in float32); the
float64 and float32 paths are timed beside it on the same plan, and the split
path's error against the float64 path is reported.

Prints one JSON line.  --gpus must be 1 (the method is shown on one GPU's
share; see the design notes for how it shards).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("RHS-transforms/s at N=16384, split-BF16 vs FP64 path @≤1e-6 rel err; %HBM BW")
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def timed_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def spmm_algorithmic_bytes(plan, R, bc, bx):
    """Bytes the banded product must move per launch: the kept entries of every
    block (bc per complex), one int32 band start per row and block, the direct
    tail (N x t reals) and its t inputs per right-hand side, the half spectra
    z_i it reads and the outputs y it writes."""
    info = plan.info()
    N, t = info["N"], info["tail"]
    spectra = sum(L // 2 + 1 for L, _, _, _ in plan.blocks())
    return (info["nnz"] * bc + 4 * N * info["n_blocks"] + N * t * bx
            + R * (t * bx + N * bx + spectra * bc))


def fft_algorithmic_bytes(plan, R, bc, bx):
    """x read once per block over its retained columns, half spectra written."""
    spectra = sum(L // 2 + 1 for L, _, _, _ in plan.blocks())
    retained = sum(hi - lo for _, _, lo, hi in plan.blocks())
    return R * (retained * bx + spectra * bc)


def cpu_baseline(w, X, rows_sample=16384):
    """The oracle's direct float64 product (A from its recurrences, then BLAS),
    timed on a sample of output rows (all of them by default) and scaled to all
    N rows."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import direct, matrix
    fam = matrix.MatrixFamily(matrix.LEGENDRE, w["N"])
    rows = np.arange(0, w["N"], w["N"] // rows_sample)[:rows_sample]
    fam.nodes()        # all nodes once (part of the oracle's setup, not timed)
    fam.weights()
    t0 = time.perf_counter()
    direct.matvec(fam, X, rows=rows)
    t = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    value = X.shape[0] / (t * w["N"] / rows.size)
    return {"value": value, "unit": "RHS-transforms/s", "cores": int(threads), "kind": "oracle",
            "sample": "direct float64 product (recurrence-built A, BLAS) on %d of %d rows, all %d "
                      "right-hand sides, %.1f s, scaled to all rows" % (rows.size, w["N"],
                                                                        X.shape[0], t)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (5 launches) and exit: "
                         "the reference reading for the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the execute path is shown on one GPU's share "
              "(right-hand sides split across GPUs need no exchange); --gpus %d is not "
              "supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.copy_mib:
        n = args.copy_mib << 18          # float32 elements
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 2.0, out=b)     # one elementwise kernel: reads a, writes b
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))
        return
    import paper_2004_11610_amd as spt
    import workloads

    w = workloads.LEGENDRE_16384
    N, R = w["N"], w["nrhs"]
    log("precompute", w["name"])
    t0 = time.perf_counter()
    plan = spt.Plan("legendre", N, w["eps"]).precompute()
    t_pre = time.perf_counter() - t0
    info = plan.info()
    log("precompute %.2f s, blocks %s, tail %d, nnz %d" % (t_pre, plan.blocks(), info["tail"],
                                                          info["nnz"]))
    Xh = workloads.rhs(w["rhs"], R, N, w["seed"])
    X64 = torch.as_tensor(Xh, device="cuda")
    X32 = X64.float()
    Y64 = torch.empty_like(X64)
    Y32 = torch.empty_like(X32)
    Ys = torch.empty_like(X32)

    paths = {"f64": (spt.F64, X64, Y64), "f32": (spt.F32, X32, Y32),
             "split_bf16": (spt.SPLIT_BF16, X32, Ys)}
    res = {}
    for name, (prec, X, Y) in paths.items():
        log("time", name)
        t = timed_steps(lambda: plan.execute(X, Y, prec=prec), args.steps, args.warmup)
        res[name] = {"ms_per_step": 1e3 * t / args.steps, "value": R * args.steps / t}
        # per-stage kernel times with HIP events on the execute stream
        spt.profile_begin()
        for _ in range(args.steps):
            plan.execute(X, Y, prec=prec)
        torch.cuda.synchronize()
        st = spt.profile_end()
        res[name]["stage_ms"] = {k: v[0] / max(v[1], 1) for k, v in st.items() if v[1]}
        log(name, res[name])
    torch.cuda.synchronize()
    y64 = Y64.cpu().numpy()
    err = {}
    for name, Y in (("f32", Y32), ("split_bf16", Ys)):
        y = Y.double().cpu().numpy()
        err[name] = float(np.max(np.linalg.norm(y - y64, axis=1) / np.linalg.norm(y64, axis=1)))
    log("errors vs f64", err)

    split = res["split_bf16"]
    spmm_ms = split["stage_ms"]["spmm"]
    bytes_spmm = spmm_algorithmic_bytes(plan, R, 8, 4)
    achieved = bytes_spmm / (spmm_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "spmm_split_bf16_kernel", "bytes_per_launch": bytes_spmm,
            "avg_launch_ms": spmm_ms}
    fft_ms = split["stage_ms"].get("fft")
    out = {
        "metric": METRIC,
        "value": split["value"],
        "unit": "RHS-transforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": split["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3",
        "data": "synthetic",
        "config": {"workload": w["name"], "family": "legendre", "N": N, "nrhs": R,
                   "eps1": w["eps"], "eps2": info["eps2"], "blocks": [b[0] for b in plan.blocks()],
                   "tail": info["tail"], "nnz": info["nnz"], "parallelism": "single-gpu"},
        "paths": {k: {"value": v["value"], "ms_per_step": v["ms_per_step"],
                      "stage_ms": v["stage_ms"]} for k, v in res.items()},
        "split_vs_f64": split["value"] / res["f64"]["value"],
        "rel_err_vs_f64": err,
        "roofline": roof,
        "fft_roofline": None if fft_ms is None else {
            "achieved": fft_algorithmic_bytes(plan, R, 8, 4) / (fft_ms * 1e-3) / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "avg_launch_ms": fft_ms},
        "precompute_s": t_pre,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, Xh)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
