#!/usr/bin/env python3
"""Benchmark of the CA-BCD s-step hot path on one MI355X.

Workload (default): dense primal ridge regression in FP64, X = U diag(sigma) V^T
with d = 2048 features, n = 262144 samples, sigma log-spaced over [1, 1e3],
lambda = 1e-4, b = 8, s = 32 (s*b = 256).  A step is one outer s-step of
CA-BCD (Alg. 2): sample the s blocks, gather the rows and form the Gram with
the residual products, the s block solves through the recurrence, and the
deferred w / residual updates.  Inputs are resident in HBM before timing.

value = algorithmic Gram flops of the timed steps (n*sb*(sb+1) per step: the
lower triangle with its diagonal) / wall time of the whole steps, in TFLOP/s.
The roofline entry times the Gram kernel alone with HIP events on the stream it
runs on.  The CPU baseline runs the FP64 oracle on a bounded number of outer
steps of the same problem on the host.

Prints one JSON line.  Single GPU only: --gpus above 1 exits with a message.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MATRIX_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--d", type=int, default=2048)
    ap.add_argument("--n", type=int, default=262144)
    ap.add_argument("--b", type=int, default=8)
    ap.add_argument("--s", type=int, default=32)
    ap.add_argument("--lam", type=float, default=1e-4)
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM bytes per Gram launch measured by rocprofv3 counters")
    return ap.parse_args()


def cpu_baseline(X, y, lam, b, s, steps, seed):
    import numpy as np
    from oracle import bcd
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    Xh = X.cpu().numpy()
    yh = y.cpu().numpy()
    stamps = []
    t0 = time.perf_counter()
    bcd.primal_bcd(Xh, yh, lam, b, s, steps * s, seed,
                   monitor=lambda h, w, z: stamps.append(time.perf_counter()))
    d, n = Xh.shape
    sb = s * b
    # per-step time from the first step's start (after the oracle's one-off
    # X^T w_0 and X y products) to the last step's end
    per_step = (stamps[-1] - t0) / steps
    flops = n * sb * (sb + 1)
    return {"value": flops / per_step / 1e12, "unit": "TFLOP/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{steps} outer steps (s={s}, b={b}) of the FP64 oracle on the same "
                      f"d={d} x n={n} problem; {per_step:.3f} s per step"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only (no collectives); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1612_04003_amd as cabcd
    import synth

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    cabcd.load()
    dev = "cuda:0"
    d, n, b, s, lam = args.d, args.n, args.b, args.s, args.lam
    sb = s * b
    seed = 2001
    print(f"[bench] generating X ({d} x {n}, FP64) on the GPU", file=sys.stderr, flush=True)
    X, y, _ = synth.spectral_ridge(d, n, 1001, device=dev)
    torch.cuda.synchronize()

    w = torch.zeros(d, dtype=torch.float64, device=dev)
    r = torch.empty(n, dtype=torch.float64, device=dev)
    print("[bench] warmup", file=sys.stderr, flush=True)
    cabcd.primal_bcd(X, y, lam, b, s, args.warmup * s, seed, w=w, r=r)
    torch.cuda.synchronize()

    tm = cabcd.new_timing()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cabcd.primal_bcd(X, y, lam, b, s, args.steps * s, seed, w=w, r=r,
                     h0=args.warmup * s, flags=cabcd.FLAG_STATE_VALID, timing=tm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    ph = cabcd.timing_dict(tm)

    gram_flops = n * sb * (sb + 1)
    value = gram_flops * args.steps / elapsed / 1e12
    g = ph["gram"]
    gram_ms = g["ms"] / max(g["launches"], 1)
    ybytes = sb * n * 8
    mfma_bound = (sb + 1) / 8.0 > PEAK_FP64_MATRIX_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    traffic = None
    try:
        with open(args.traffic_json) as fh:
            tj = json.load(fh)
        key = f"gram_f64_d{d}_n{n}_sb{sb}"
        traffic = tj.get(key)
    except (OSError, ValueError):
        pass
    if mfma_bound:
        achieved = gram_flops / (gram_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64_MATRIX_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_MATRIX_TFLOPS, 4),
                "traffic": traffic}
    else:
        achieved = ybytes / (gram_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic}
    roof["kernel"] = "gram_f64_kernel<16>" if sb > 128 else "gram_f64_kernel"
    roof["per_launch"] = {"flops": gram_flops, "bytes": ybytes, "ms": round(gram_ms, 4)}

    out = {
        "metric": "CA-BCD Gram TFLOP/s (% peak) + time-to-1e-6 rel obj error, FP64 vs mixed",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"dense primal CA-BCD ridge, FP64, d={d} n={n} "
                               f"spectrum 1..1e3, lambda={lam:g}, b={b}, s={s}",
                   "d": d, "n": n, "b": b, "s": s, "lambda": lam, "sb": sb},
        "roofline": roof,
        "phases_ms_per_step": {k: round(v["ms"] / args.steps, 4) for k, v in ph.items()
                               if v["launches"]},
    }
    if not args.no_cpu_baseline:
        print("[bench] CPU baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(X, y, lam, b, s, args.cpu_steps, seed)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
