#!/usr/bin/env python3
"""Throughput of the extra-component computation stage on one MI355X.

Workload: the Legendre transform of order N = 16384 (orthonormalised, Gauss-
Legendre nodes), 64 right-hand sides x ~ N(0, 1) (seed 1), eps1 = 1e-7,
eps2 = 1e-2, float64 precomputation.  One step = one spt_execute of all 64
right-hand sides (extend + window + FFT of every block, banded product of every
block and the direct tail): two launches, the FFTs of every block, then the
banded products.  The timed steps are dealt in turn to --streams streams
(default 3; four measured the same for the split path and about 10% slower
for float64, with the runtime's four hardware queues per process), each with
its own output buffer, so that independent batches are in flight together as
in serving; the one-stream rate (each step after the
previous one) is reported beside it.  The headline value is the split-bf16 path (float32 FFT,
three-piece bfloat16 matrix-core product accumulated in float32); the float64
and float32 paths are timed beside it on the same plan, the split path's error
against the float64 path is reported, and the one-launch persistent executor
is timed on the same workload for comparison.

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


def algorithmic_bytes(plan, R, bc, bx):
    """Bytes the whole computation stage must move for R right-hand sides: the
    kept entries of every block (bc per complex), one int32 band start per row
    and block, the direct tail (N x t reals), x read and y written once, and the
    half spectra z_i written by the FFTs and read back by the products."""
    info = plan.info()
    N, t = info["N"], info["tail"]
    spectra = sum(L // 2 + 1 for L, _, _, _ in plan.blocks())
    return (info["nnz"] * bc + 4 * N * info["n_blocks"] + N * t * bx
            + R * (N * bx + N * bx + 2 * spectra * bc))


def fft_bytes(plan, R, bc, bx, blocks=None):
    """Bytes of an FFT launch over `blocks` (default all): each block reads its
    retained columns of x and writes its half spectrum."""
    bl = plan.blocks()
    idx = range(len(bl)) if blocks is None else blocks
    spectra = sum(bl[i][0] // 2 + 1 for i in idx)
    retained = sum(bl[i][3] - bl[i][2] for i in idx)
    return R * (retained * bx + spectra * bc)


def product_bytes(plan, R, bc, bx, blocks=None, tail=True):
    """Bytes of a banded-product launch over `blocks` (default all): their kept
    entries and band starts, the tail and its x columns when `tail`, the half
    spectra read, y written."""
    info = plan.info()
    N, t = info["N"], (info["tail"] if tail else 0)
    bl = plan.blocks()
    idx = list(range(len(bl))) if blocks is None else list(blocks)
    spectra = sum(bl[i][0] // 2 + 1 for i in idx)
    nnz = sum(info["nnz_blk"][i] for i in idx)
    return (nnz * bc + 4 * N * len(idx) + N * t * bx
            + R * (t * bx + N * bx + spectra * bc))


KERNEL_SOURCES = ("fft.hip", "spmm.hip", "fft_core.hpp", "spmm_core.hpp", "common.hpp")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2004_11610_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's reading), if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "%s_legendre_n16384_r64.md" % kernel)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel sources sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, X, rows_sample=16384, compressed_leg=True):
    """The oracle's direct float64 product (A from its recurrences, then BLAS),
    timed on a sample of output rows (all of them by default) and scaled to all
    N rows; beside it, the oracle's compressed method on the same plan."""
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
    out = {"value": value, "unit": "RHS-transforms/s", "cores": int(threads), "kind": "oracle",
           "sample": "direct float64 product (recurrence-built A, BLAS) on %d of %d rows, all %d "
                     "right-hand sides, %.1f s, scaled to all rows" % (rows.size, w["N"],
                                                                       X.shape[0], t)}
    if compressed_leg:
        # the oracle's compressed method (full spectrum, scipy.sparse): its
        # precomputation once (not part of the rate), then executes of all the
        # right-hand sides
        from oracle import compressed
        t0 = time.perf_counter()
        comp = compressed.Compressed(compressed.Plan(fam, w["eps"], 1e-2))
        t_pre = time.perf_counter() - t0
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            comp.execute(X)
        t = (time.perf_counter() - t0) / reps
        out["compressed"] = {"value": X.shape[0] / t, "unit": "RHS-transforms/s",
                             "cores": int(threads), "precompute_s": t_pre,
                             "sample": "the oracle's compressed method (numpy FFTs, scipy.sparse "
                                       "product), all %d rows and %d right-hand sides, mean of "
                                       "%d executes" % (w["N"], X.shape[0], reps)}
    return out


def large_workload(args, spt, workloads):
    """The 48-plan batch (one staged batch per step, all plans) or the
    Laguerre-function plan (N = 65536, 1024 right-hand sides): float64 and
    split-bf16 throughput in RHS-transforms/s (sum of right-hand sides over
    the step time)."""
    import numpy as np
    import torch
    fams = {2: "legendre", 3: "jacobi", 4: "laguerre_fn", 5: "hermite_fn"}
    ws = workloads.batch_plans() if args.workload == "batch48" else [workloads.LAGUERRE_65536]
    prec_mask = (1 << spt.F64) | (1 << spt.SPLIT_BF16)
    t0 = time.perf_counter()
    plans = [spt.Plan(fams[w["family"]], w["N"], w["eps"], alpha=w.get("alpha", 0.0),
                      beta=w.get("beta", 0.0), precisions=prec_mask).precompute() for w in ws]
    t_pre = time.perf_counter() - t0
    log("precompute %d plans %.1f s" % (len(plans), t_pre))
    Xh = [workloads.rhs(w["rhs"], w["nrhs"], w["N"], w["seed"]) for w in ws]
    total_r = sum(w["nrhs"] for w in ws)
    out = {"metric": "RHS-transforms/s", "workload": args.workload, "plans": len(ws),
           "nrhs_total": total_r, "precompute_s": t_pre,
           "modes": [p.info()["mode"] for p in plans], "paths": {}}
    for name, prec, dt in (("f64", spt.F64, torch.float64), ("split_bf16", spt.SPLIT_BF16,
                                                             torch.float32)):
        X = [torch.as_tensor(x, device="cuda").to(dt) for x in Xh]
        Y = [torch.empty_like(x) for x in X]
        run = lambda: spt.execute_batched(plans, X, Y, prec=prec)
        steps = max(3, min(args.steps, 20))
        t = timed_steps(run, steps, min(args.warmup, 3))
        spt.profile_begin()
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        st = spt.profile_end()
        out["paths"][name] = {"value": total_r * steps / t, "ms_per_step": 1e3 * t / steps,
                              "kernel_ms": {k: v[0] / max(v[1], 1) for k, v in st.items() if v[1]}}
        # matrix-core work of the product as issued: every stored box entry
        # (complex, zeros inside the boxes included) times every right-hand
        # side, 4 flop each (Re a Re z - Im a Im z), six piece products in
        # split-bf16
        km = out["paths"][name]["kernel_ms"].get("spmm")
        if km:
            flop = sum(p.info()["stored"] * w["nrhs"] for p, w in zip(plans, ws)) * 4.0
            flop *= 6.0 if name == "split_bf16" else 1.0
            peak = 2500.0 if name == "split_bf16" else 78.6
            out["paths"][name]["product_tflops"] = flop / (km * 1e-3) / 1e12
            out["paths"][name]["product_mfma_frac"] = flop / (km * 1e-3) / 1e12 / peak
        log(name, out["paths"][name])
        del X, Y
    return out


def generators_workload(args, spt, workloads):
    """The other generators the method takes (sec. 2, eq. cosd2, sec. 4.1) and
    the Appendix A precompute, at the benchmark's 64 right-hand sides: one
    stream, executes back to back; per path the RHS-transforms/s, the stage
    times (HIP events) and the relative error against float64."""
    import numpy as np
    import torch
    R = 64
    cases = [("sine-n16384", "sine", 16384, {}),
             ("cos3-n16384", "cos_power", 16384, dict(power=3)),
             ("chebyshev-n16384-appendix-a", "chebyshev_t", 16384, dict(trig_conv_q=12)),
             ("cexp-n4096", "cexp", 4096, {}),
             ("laguerre-spectral-n4096", "laguerre_spectral", 4096,
              dict(eta=100.0, period=4.0))]
    out = {"metric": "RHS-transforms/s", "workload": "generators", "nrhs": R, "eps1": 1e-7,
           "plans": {}}
    steps = max(10, min(args.steps, 100))
    for name, fam, N, kw in cases:
        cplx = fam in ("cexp", "laguerre_spectral")
        t0 = time.perf_counter()
        p = spt.Plan(fam, N, 1e-7, **kw).precompute()
        torch.cuda.synchronize()
        res = {"N": N, "precompute_s": time.perf_counter() - t0, "blocks": [b[0] for b in p.blocks()],
               "nnz": p.info()["nnz"], "stored": p.info()["stored"], "paths": {}}
        if fam == "chebyshev_t":
            t0 = time.perf_counter()
            q = spt.Plan(fam, N, 1e-7).precompute()
            torch.cuda.synchronize()
            res["precompute_row_ffts_s"] = time.perf_counter() - t0
            q.close()
        g = np.random.default_rng(77)
        Xh = g.standard_normal((R, N)) + (1j * g.standard_normal((R, N)) if cplx else 0.0)
        precs = [("f64", spt.F64), ("f32", spt.F32)] + ([] if cplx else [("split_bf16", spt.SPLIT_BF16)])
        ref = {}
        for tr in (False, True):
            for pname, prec in precs:
                if tr and prec == spt.SPLIT_BF16:
                    continue
                dt = (torch.complex128 if prec == spt.F64 else torch.complex64) if cplx else \
                     (torch.float64 if prec == spt.F64 else torch.float32)
                X = torch.as_tensor(Xh).to(device="cuda", dtype=dt)
                f = p.execute_transposed if tr else p.execute
                Y = f(X, prec=prec)
                run = lambda: f(X, Y, prec=prec)
                t = timed_steps(run, steps, 5)
                spt.profile_begin()
                for _ in range(steps):
                    run()
                torch.cuda.synchronize()
                st = spt.profile_end()
                key = ("transposed_" if tr else "") + pname
                y = Y.cpu().numpy().astype(np.complex128 if cplx else np.float64)
                if prec == spt.F64:
                    ref[tr] = y
                err = float(np.max(np.linalg.norm(y - ref[tr], axis=1) /
                                   np.linalg.norm(ref[tr], axis=1)))
                res["paths"][key] = {"value": R * steps / t, "ms_per_execute": 1e3 * t / steps,
                                     "kernel_ms": {k: v[0] / max(v[1], 1) for k, v in st.items()
                                                   if v[1]},
                                     "rel_err_vs_f64": err}
                log(name, key, res["paths"][key])
        out["plans"][name] = res
        p.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-compressed", action="store_true",
                    help="skip the oracle's compressed method in the CPU baseline (its "
                         "precomputation takes about a minute)")
    ap.add_argument("--streams", type=int, default=3,
                    help="streams the timed steps are dealt to in turn (independent "
                         "batches in flight at once; 1 = strictly one after another)")
    ap.add_argument("--workload", default="legendre-n16384-r64",
                    choices=["legendre-n16384-r64", "batch48", "laguerre-fn-n65536-r1024",
                             "generators"],
                    help="the headline workload (default), one of the two large ones "
                         "(timed the same way), or the other generators and the Appendix A "
                         "precompute (reported for the design notes)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch choices instead of spt_autotune's")
    ap.add_argument("--tuning", default="",
                    help="launch choices to use instead of the autotuner's, e.g. "
                         "product=2,window_rhs=32,fft_batch=4 (spt_tuning fields)")
    ap.add_argument("--reduced-fft", type=int, default=0, choices=[0, 1, 2],
                    help="arithmetic of the float32 paths' FFTs: 0 chosen by the plan "
                         "(spt_params.reduced_fft), 1 float32, 2 float64")
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
    if args.workload == "generators":
        print(json.dumps(generators_workload(args, spt, workloads)), flush=True)
        return
    if args.workload != "legendre-n16384-r64":
        print(json.dumps(large_workload(args, spt, workloads)), flush=True)
        return

    w = workloads.LEGENDRE_16384
    N, R = w["N"], w["nrhs"]
    log("precompute", w["name"])
    t0 = time.perf_counter()
    plan = spt.Plan("legendre", N, w["eps"], reduced_fft=args.reduced_fft).precompute()
    t_pre = time.perf_counter() - t0
    info = plan.info()
    log("precompute %.2f s, blocks %s, tail %d, nnz %d" % (t_pre, plan.blocks(), info["tail"],
                                                          info["nnz"]))
    # launch choices by the library's autotuner (timed on the split-bf16 path;
    # the float64 and float32 paths run with the same choices)
    tuning = {"autotuned": False}
    if args.tuning:
        plan.set_tuning(**{k: int(v) for k, v in (kv.split("=") for kv in args.tuning.split(","))})
        tuning = dict(plan.tuning(), autotuned=False)
    elif not args.no_autotune:
        t0 = time.perf_counter()
        chosen, us = plan.autotune(R, prec=spt.SPLIT_BF16)
        tuning = dict(chosen, autotuned=True, us_per_execute=us,
                      seconds=time.perf_counter() - t0)
        log("autotune", tuning)
    Xh = workloads.rhs(w["rhs"], R, N, w["seed"])
    X64 = torch.as_tensor(Xh, device="cuda")
    X32 = X64.float()
    Y64 = torch.empty_like(X64)
    Y32 = torch.empty_like(X32)
    Ys = torch.empty_like(X32)

    paths = {"f64": (spt.F64, X64, Y64), "f32": (spt.F32, X32, Y32),
             "split_bf16": (spt.SPLIT_BF16, X32, Ys)}
    res = {}

    def measure(pl, prec, X, Y, transposed=False):
        # steps dealt to the streams in turn: each step is a whole execute of
        # the 64 right-hand sides into its stream's output buffer
        run = pl.execute_transposed if transposed else pl.execute
        streams = [torch.cuda.Stream() for _ in range(args.streams)]
        Ys = [Y] + [torch.empty_like(Y) for _ in range(args.streams - 1)]
        state = {"i": 0}

        # each execute names its stream (no stream context per step: entering
        # one costs the host more than a step's launches)
        def step():
            j = state["i"] % args.streams
            state["i"] += 1
            run(X, Ys[j], prec=prec, stream=streams[j])

        torch.cuda.synchronize()
        t = timed_steps(step, args.steps, args.warmup)
        s0 = torch.cuda.current_stream()
        t1 = timed_steps(lambda: run(X, Y, prec=prec, stream=s0), args.steps, args.warmup)
        r = {"ms_per_step": 1e3 * t / args.steps, "value": R * args.steps / t,
             "streams": args.streams,
             "one_stream": {"ms_per_step": 1e3 * t1 / args.steps, "value": R * args.steps / t1}}
        # kernel times with HIP events on the execute stream
        spt.profile_begin()
        for _ in range(args.steps):
            run(X, Y, prec=prec)
        torch.cuda.synchronize()
        st = spt.profile_end()
        r["kernel_ms"] = {k: v[0] / max(v[1], 1) for k, v in st.items() if v[1]}
        return r

    for name, (prec, X, Y) in paths.items():
        log("time", name)
        res[name] = measure(plan, prec, X, Y)
        log(name, res[name])
    torch.cuda.synchronize()
    y64 = Y64.cpu().numpy()
    err = {}
    for name, Y in (("f32", Y32), ("split_bf16", Ys)):
        y = Y.double().cpu().numpy()
        err[name] = float(np.max(np.linalg.norm(y - y64, axis=1) / np.linalg.norm(y64, axis=1)))
    log("errors vs f64", err)
    # the transposed product (Alg. 2/4) on the same plan and inputs
    res_t = {}
    for name in ("f64", "f32"):
        prec, X, Y = paths[name]
        log("time transposed", name)
        res_t[name] = measure(plan, prec, X, torch.empty_like(Y), transposed=True)
        log("transposed", name, res_t[name])
    # cold caches: before every timed execute a 1 GiB buffer is written, which
    # evicts the L2s and the 256 MB Infinity Cache; the execute (HIP events on
    # its stream) then reads the plan and x from HBM
    log("cold-cache executes")
    cold = {}
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    for name, (prec, X, Y) in paths.items():
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(20)]
        for a, b in ev:
            flush.fill_(1.0)
            a.record()
            plan.execute(X, Y, prec=prec)
            b.record()
        torch.cuda.synchronize()
        ms = sorted(a.elapsed_time(b) for a, b in ev)
        med = ms[len(ms) // 2]
        cold[name] = {"ms_per_execute": med, "value": R / (med * 1e-3),
                      "note": "median of 20 executes, each after a 1 GiB write"}
    del flush
    log("cold", cold)
    # the one-launch persistent executor on the same workload, for comparison
    pers = spt.Plan("legendre", N, w["eps"], executor=spt.EXECUTOR_PERSISTENT).precompute()
    log("time split_bf16, persistent executor")
    Yp = torch.empty_like(X32)
    res_pers = measure(pers, spt.SPLIT_BF16, X32, Yp)
    log("persistent", res_pers)
    pers.close()

    split = res["split_bf16"]
    km = split["kernel_ms"]
    # the two launches of the split-bf16 step.  Algorithmic bytes count the
    # method's data at the path's precision: 8 bytes per complex value of the
    # compressed blocks and of the half spectra, 4 per real of x and y.  The
    # library's layout stores both as three bfloat16 pieces (12 bytes per
    # complex value); those bytes are reported as layout_bytes_per_launch, and
    # what HBM actually moved as traffic (rocprofv3 counters).
    spmm_kernel = "spmm_window_kernel" if info["window_lds"] > 0 else "spmm_presplit_kernel"
    fft_kernel = ("exec_fft_multi_kernel<double, float, true>" if info["reduced_fft_f64"]
                  else "exec_fft_multi_kernel<float, float, true>")
    launches = {"fft": (fft_kernel, fft_bytes(plan, R, 8, 4),
                        fft_bytes(plan, R, 12, 4)),
                "spmm": (spmm_kernel, product_bytes(plan, R, 8, 4),
                         product_bytes(plan, R, 12, 4))}

    def roofline(stage):
        name, nbytes, layout = launches[stage]
        achieved = nbytes / (km[stage] * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(stage),
                "kernel": name, "bytes_per_launch": nbytes, "layout_bytes_per_launch": layout,
                "avg_launch_ms": km[stage]}

    dominant = max(launches, key=lambda k: km.get(k, 0.0))
    roof = roofline(dominant)
    other = {k: roofline(k) for k in launches if k != dominant}
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
                   "tail": info["tail"], "nnz": info["nnz"], "stored": info["stored"],
                   "parallelism": "single-gpu",
                   "reduced_fft_f64": info["reduced_fft_f64"],
                   "reduced_fft_f32_err": info["reduced_fft_f32_err"], "tuning": tuning},
        "streams": args.streams,
        "paths": {k: {"value": v["value"], "ms_per_step": v["ms_per_step"],
                      "one_stream": v["one_stream"], "kernel_ms": v["kernel_ms"]}
                  for k, v in res.items()},
        "split_bf16_persistent_executor": {"value": res_pers["value"],
                                           "ms_per_step": res_pers["ms_per_step"],
                                           "one_stream": res_pers["one_stream"],
                                           "kernel_ms": res_pers["kernel_ms"]},
        "transposed": {k: {"value": v["value"], "ms_per_step": v["ms_per_step"],
                           "one_stream": v["one_stream"], "kernel_ms": v["kernel_ms"]}
                       for k, v in res_t.items()},
        "split_vs_f64": split["value"] / res["f64"]["value"],
        "rel_err_vs_f64": err,
        "roofline": roof,
        "roofline_other_launches": other,
        "stage_bytes_per_step": algorithmic_bytes(plan, R, 8, 4),
        "cold": cold,
        "kernel_sources_sha256": kernel_source_hash(),
        "precompute_s": t_pre,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, Xh, compressed_leg=not args.no_cpu_compressed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
