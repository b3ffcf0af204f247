#!/usr/bin/env python3
"""Benchmark of the CA-BCD s-step hot path on one MI355X.

Headline workload: dense primal ridge regression in FP64, X = U diag(sigma) V^T
with d = 2048 features, n = 262144 samples, sigma log-spaced over [1, 1e3],
lambda = 1e-4, b = 8, s = 32 (s*b = 256).  A step is one outer s-step of
CA-BCD (Alg. 2): sample the s blocks, gather the rows and form the Gram with
the residual products, the s block solves through the recurrence, and the
deferred w / residual updates.  Inputs are resident in HBM before timing.

value = algorithmic Gram flops of the timed steps (n*sb*(sb+1) per step: the
lower triangle with its diagonal) / wall time of the whole steps, in TFLOP/s.
roofline: the Gram kernel alone, timed with HIP events on the stream it runs
on.  folded_update: the same steps with CABCD_FLAG_FOLD_UPDATE (each step's
residual update applied inside the next step's Gram kernel).  cpu_baseline: the FP64 oracle on a bounded number of outer steps of the
same problem on the host.

time_to_tol: wall time from the first s-step until a monitor point (every 4
outer steps, each with an exact residual recomputation) shows a relative
objective error <= 1e-6, on the column-scaled workload d = 4096, n = 2^20,
lambda = 1e-4, b = 16, s = 16: FP64 CA-BCD on the dequantised matrix X^ versus
the mixed-precision runs on the BF16 / FP8 storage of the same X^.

extra: shorter records of the other configurations (s sweep of the headline,
the dense dual on X^T, the sparse dual on a Zipf CSR matrix).

Prints one JSON line on stdout (progress goes to stderr).  Single GPU only.
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


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


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
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--settle", type=float, default=0.1,
                    help="seconds of untimed outer steps before the warm-up (clock ramp)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tol", action="store_true", help="skip the time-to-1e-6 runs")
    ap.add_argument("--no-extra", action="store_true", help="skip the extra records")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched time-to-1e-6 runs")
    ap.add_argument("--only-batch", action="store_true", help="run only the batched record")
    ap.add_argument("--batch-no-baseline", action="store_true",
                    help="batched record without the one-problem-at-a-time baseline")
    ap.add_argument("--only-tol", action="store_true", help="run only the mixed time-to-1e-6")
    ap.add_argument("--only-extra", action="store_true",
                    help="run only the extra records (s sweep, dual, sparse, residual stops)")
    ap.add_argument("--no-stability", action="store_true",
                    help="skip the numerical-stability record")
    ap.add_argument("--only-sparse", action="store_true",
                    help="run only the sparse dual records (CSR, s = 1, 8, 32)")
    ap.add_argument("--only-stability", action="store_true",
                    help="run only the numerical-stability record")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB of FP64 three times (the reference kernel that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters to bytes)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM bytes per Gram launch measured by rocprofv3 counters")
    return ap.parse_args()


def cpu_baseline(X, y, lam, b, s, steps, seed):
    """The FP64 oracle on the host cores, with the paper's timing protocol (one
    warm-up run and three timed runs, mean and minimum): each run is `steps`
    outer steps of the headline problem, once with the matrix library on one
    thread and once on every thread it has.  value is the all-thread mean."""
    from oracle import bcd
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    Xh = X.cpu().numpy()
    yh = y.cpu().numpy()
    d, n = Xh.shape
    sb = s * b
    flops = n * sb * (sb + 1) * steps

    def protocol(limit):
        times = []
        with threadpool_limits(limits=limit):
            for _ in range(4):
                t0 = time.perf_counter()
                bcd.primal_bcd(Xh, yh, lam, b, s, steps * s, seed)
                times.append(time.perf_counter() - t0)
        return times[1:]

    t_all = protocol(threads)
    t_one = protocol(1)
    mean_all, mean_one = sum(t_all) / 3, sum(t_one) / 3
    log(f"cpu baseline: {threads} threads {t_all}, 1 thread {t_one}")
    return {"value": flops / mean_all / 1e12, "unit": "TFLOP/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{steps} outer steps (s={s}, b={b}) of the FP64 oracle on the same "
                      f"d={d} x n={n} problem per run; 1 warm-up + 3 timed runs; "
                      f"{mean_all / steps:.3f} s per step on {threads} threads, "
                      f"{mean_one / steps:.3f} s on 1",
            "runs_s": [round(t, 4) for t in t_all],
            "best": flops / min(t_all) / 1e12,
            "single_thread": {"value": flops / mean_one / 1e12, "cores": 1,
                              "runs_s": [round(t, 4) for t in t_one],
                              "best": flops / min(t_one) / 1e12}}


def closed_form(cabcd, torch, X, y, lam):
    """The ridge minimiser (X X^T / n + lam I) w = X y / n on the GPU (Cholesky of
    the d x d normal matrix in FP64) and f(w*) by the library's objective.
    Reference values outside every timed region; the GPU tests check this
    routine against the oracle's closed form."""
    n = X.shape[1]
    M = X @ X.t()
    M /= n
    M.diagonal().add_(lam)
    L = torch.linalg.cholesky(M)
    del M
    w = torch.cholesky_solve(((X @ y) / n)[:, None], L)[:, 0]
    del L
    f, _ = cabcd.primal_objective(X, y, lam, w)
    return w, f.item()


def timed_primal(cabcd, torch, X, y, lam, b, s, steps, warmup, seed, dual=False, mask=0,
                 settle_s=0.0, flags=0):
    """Warm up, then time `steps` outer steps; returns (elapsed s, phase dict).
    `mask` selects the phases bracketed by HIP events (0: all); every event
    pair costs GPU time, so the timed headline run brackets the Gram only.
    settle_s > 0: before the `warmup` steps, untimed outer steps run until the
    GPU has been busy that long: coming out of idle, the GPU's clocks take
    some 20 ms of load to ramp up (the first 20 steps of the headline run 15 %
    slower than the steady state of a long solve)."""
    rows, cols = X.shape
    coord = torch.zeros(rows, dtype=torch.float64, device=y.device)
    comp = torch.empty(cols, dtype=torch.float64, device=y.device)
    run = cabcd.dual_bcd if dual else cabcd.primal_bcd
    if dual:
        kw0 = dict(alpha=coord, w=comp)
    else:
        kw0 = dict(w=coord, r=comp)
    if settle_s > 0.0:
        t_end = time.perf_counter() + settle_s
        while time.perf_counter() < t_end:
            run(X, y, lam, b, s, 10 * s, seed, flags=flags, **kw0)
            torch.cuda.synchronize()
        coord.zero_()
    run(X, y, lam, b, s, warmup * s, seed, flags=flags, **kw0)
    torch.cuda.synchronize()
    tm = cabcd.new_timing()
    t0 = time.perf_counter()
    run(X, y, lam, b, s, steps * s, seed, h0=warmup * s, flags=cabcd.FLAG_STATE_VALID | flags,
        timing=tm, timing_mask=mask, **kw0)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, cabcd.timing_dict(tm)


def measured_traffic(path, key):
    """HBM bytes per launch from the committed PMC summary, or None when there is
    none for this workload or the kernel sources changed since it was taken."""
    import hashlib
    try:
        with open(path) as fh:
            ent = json.load(fh).get(key)
        if ent is None:
            return None
        h = hashlib.sha256()
        for f in ent["sources"]:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        return ent["bytes"] if h.hexdigest()[:16] == ent["sources_sha256_16"] else None
    except (OSError, ValueError, KeyError):
        return None


def padded(cabcd, X):
    """X (rows x cols, FP64) copied into rows leading_dim(cols) apart: the same
    matrix in the layout the library recommends (a 2 MiB row stride, as
    contiguous rows of 2^18 columns have, sends the gathered rows' same
    columns to the same HBM channels)."""
    Y = cabcd.empty_dense(X.shape[0], X.shape[1], X.device)
    Y.copy_(X)
    return Y


def headline(args, cabcd, torch, synth):
    dev = "cuda:0"
    d, n, b, s, lam = args.d, args.n, args.b, args.s, args.lam
    sb = s * b
    log(f"generating X ({d} x {n}, FP64) on the GPU")
    X, y, _ = synth.spectral_ridge(d, n, 1001, device=dev)
    X = padded(cabcd, X)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    gram_only = 1 << cabcd.PHASES.index("gram")
    elapsed, ph = timed_primal(cabcd, torch, X, y, lam, b, s, args.steps, args.warmup, 2001,
                               mask=gram_only, settle_s=args.settle)
    log("phase breakdown run (every phase bracketed by events)")
    _, ph_all = timed_primal(cabcd, torch, X, y, lam, b, s, min(args.steps, 10), 1, 2001)
    gram_flops = n * sb * (sb + 1)
    value = gram_flops * args.steps / elapsed / 1e12
    g = ph["gram"]
    gram_ms = g["ms"] / max(g["launches"], 1)
    ybytes = sb * n * 8
    mfma_bound = (sb + 1) / 8.0 > PEAK_FP64_MATRIX_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    traffic = measured_traffic(args.traffic_json, f"gram_f64_d{d}_n{n}_sb{sb}")
    if mfma_bound:
        achieved = gram_flops / (gram_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64_MATRIX_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_MATRIX_TFLOPS, 4),
                "traffic": traffic}
    else:
        achieved = ybytes / (gram_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic}
    roof["kernel"] = ("gram_f64_dma16_kernel" if sb > 128 and n % 2 == 0 else
                      "gram_f64_kernel<16,2>" if sb > 128 else "gram_f64_kernel")
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
        # from a separate 10-step run with every phase bracketed by events (the
        # events add a few microseconds per phase, so these sum to more than
        # ms_per_step)
        "phases_ms_per_step": {k: round(v["ms"] / min(args.steps, 10), 4)
                               for k, v in ph_all.items() if v["launches"]},
    }
    if sb == 256 and n % 2 == 0:
        # the same steps with each step's residual update applied inside the
        # next step's Gram kernel: that kernel streams the previous step's
        # rows too (its bytes 2 sb n 8 + 16 n), the step skips its update pass
        log("timing the steps with the update folded into the next Gram")
        el_f, ph_f = timed_primal(cabcd, torch, X, y, lam, b, s, args.steps, args.warmup, 2001,
                                  mask=gram_only, flags=cabcd.FLAG_FOLD_UPDATE)
        gf = ph_f["gram"]
        gf_ms = gf["ms"] / max(gf["launches"], 1)
        out["folded_update"] = {
            "ms_per_step": round(el_f / args.steps * 1e3, 4),
            "value": round(gram_flops * args.steps / el_f / 1e12, 3),
            "kernel": "gram_f64_dma16_upd_kernel<1> (the call's first step: gram_f64_dma16_kernel)",
            "gram_ms": round(gf_ms, 4),
            "gram_frac": round(gram_flops / (gf_ms * 1e-3) / 1e12 / PEAK_FP64_MATRIX_TFLOPS, 4),
            "gram_bytes": 2 * ybytes + 16 * n}
    return out, X, y


def extra_records(args, cabcd, torch, synth, X, y):
    """Other shapes of the path (events bracket the Gram only; the event pair
    costs a few microseconds per step, which shows at s = 1: graph_small_steps
    has the small steps without events); per_iteration_us = step time / s, the
    cost of one b-coordinate iteration, shows what the s-step form saves."""
    rec = {}
    gram_only = 1 << cabcd.PHASES.index("gram")
    d, n, lam = args.d, args.n, args.lam
    for s in (1, 4, 16):
        sb = s * args.b
        el, ph = timed_primal(cabcd, torch, X, y, lam, args.b, s, 20, 2, 2001, mask=gram_only)
        g = ph["gram"]["ms"] / 20   # Gram time per outer step
        rec[f"primal_s{s}"] = {"ms_per_step": round(el / 20 * 1e3, 4),
                               "per_iteration_us": round(el / 20 / s * 1e6, 2),
                               "gram_ms": round(g, 4),
                               "gram_tflops": round(n * sb * (sb + 1) / (g * 1e-3) / 1e12, 3),
                               "gram_gbs": round(sb * n * 8 / (g * 1e-3) / 1e9, 1)}
        log(f"primal s={s}: {rec[f'primal_s{s}']}")
    XT = X.t().contiguous()
    for s in (1, 4, 16, 32):
        el, ph = timed_primal(cabcd, torch, XT, y, lam, args.b, s, 20, 2, 2001, dual=True,
                              mask=gram_only)
        g = ph["gram"]["ms"] / 20
        sb = s * args.b
        rec[f"dual_s{s}"] = {"ms_per_step": round(el / 20 * 1e3, 4),
                             "per_iteration_us": round(el / 20 / s * 1e6, 2),
                             "gram_ms": round(g, 4),
                             "gram_tflops": round(d * sb * (sb + 1) / (g * 1e-3) / 1e12, 3)}
        log(f"dual s={s}: {rec[f'dual_s{s}']}")
    del XT
    sp, A, yd = sparse_records(cabcd, torch, synth)
    rec.update(sp)
    rec.update(resid_tol_records(cabcd, torch, X, y, lam, args.b, args.s, A, yd))
    rec["graph_small_steps"] = graph_records(cabcd, torch, X, y, lam)
    return rec


def sparse_records(cabcd, torch, synth):
    """Sparse dual on A = X^T in CSR, 20000 rows x 2^20 columns, 315 Zipf(1.1)
    features per row, b = 16, s = 1, 8, 32."""
    import numpy as np
    rec = {}
    gram_only = 1 << cabcd.PHASES.index("gram")
    log("generating the sparse problem (CSR, 20000 x 2^20)")
    rowptr, colidx, vals, ys, _ = synth.zipf_csr_ridge(20000, 1 << 20, 315, 1002)
    A = cabcd.CSR(torch.tensor(rowptr, device="cuda"), torch.tensor(colidx, device="cuda"),
                  torch.tensor(vals, device="cuda"), (20000, 1 << 20))
    yd = torch.tensor(ys, device="cuda")
    steps = 32   # two whole launches of the split Gram (16 steps each) at s b >= 256
    for s in (1, 8, 32):
        b = 16
        el, ph = timed_primal(cabcd, torch, A, yd, 1e-5, b, s, steps, 2, 2002, dual=True,
                              mask=gram_only)
        # per outer step: the Grams of several future steps come from one launch,
        # the Y u of each step from its own
        g = ph["gram"]["ms"] / steps
        # algorithmic Gram work of the sampled rows: 2 sum_c nnz_c(I)^2 flops over the
        # nnz of the gathered rows (12 bytes each), averaged over the timed steps
        idx = cabcd.sample(2002, 2 * s, steps * s, b, 20000).cpu().numpy().reshape(steps, s * b)
        fl, by = [], []
        for blk in idx:
            cols = np.concatenate([colidx[rowptr[i]:rowptr[i + 1]] for i in blk])
            cnt = np.bincount(cols)
            fl.append(2.0 * float((cnt.astype(np.float64) ** 2).sum()))
            by.append(12.0 * len(cols))
        rec[f"sparse_dual_s{s}"] = {
            "ms_per_step": round(el / steps * 1e3, 4), "gram_ms": round(g, 4),
            "gram_gflops": round(np.mean(fl) / (g * 1e-3) / 1e9, 2),
            "gram_gbs": round(np.mean(by) / (g * 1e-3) / 1e9, 2)}
        log(f"sparse dual s={s}: {rec[f'sparse_dual_s{s}']}")
    return rec, A, yd


def graph_records(cabcd, torch, X, y, lam, steps=64):
    """Small outer steps with and without HIP graph capture: one call of
    `steps` outer steps timed as issued (launches from the host), against the
    same call captured once into a graph (caller workspace, no synchronisation
    inside the call) and replayed.  Each replay repeats the captured
    iterations from the state it finds; both rates are per outer step on the
    headline matrix."""
    out = {}
    d, n = X.shape
    for (b, s) in ((8, 1), (1, 1), (1, 8), (8, 4)):
        ws = torch.empty(cabcd.workspace_bytes(X, b, s), dtype=torch.uint8, device="cuda")
        w = torch.zeros(d, dtype=torch.float64, device="cuda")
        r = torch.empty(n, dtype=torch.float64, device="cuda")
        H = steps * s
        kw = dict(w=w, r=r, workspace=ws)
        cabcd.primal_bcd(X, y, lam, b, s, H, 77, **kw)
        flags = cabcd.FLAG_STATE_VALID | cabcd.FLAG_ASYNC
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            cabcd.primal_bcd(X, y, lam, b, s, H, 77, h0=H, flags=flags, **kw)
        torch.cuda.synchronize()
        direct = (time.perf_counter() - t0) / (3 * steps)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            cabcd.primal_bcd(X, y, lam, b, s, H, 77, h0=H, flags=flags, **kw)
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        graph = (time.perf_counter() - t0) / (3 * steps)
        out[f"b{b}s{s}"] = {"direct_us_per_step": round(direct * 1e6, 2),
                            "graph_us_per_step": round(graph * 1e6, 2),
                            "direct_us_per_iteration": round(direct * 1e6 / s, 2),
                            "graph_us_per_iteration": round(graph * 1e6 / s, 2)}
        log(f"graph b={b} s={s}: {out[f'b{b}s{s}']}")
        del g, ws
    return out


def resid_tol_records(cabcd, torch, X, y, lam, b, s, A, yd, every=8):
    """Runs stopped by the residual test of Section 5.1.5 (tolerances of the
    paper's performance runs: 1e-1 primal, 1e-2 dual, relative to the
    residual at the start): wall time, inner iterations, and the cost of one
    check (a full pass over A) from a second, event-timed run."""
    rec = {}
    dev = X.device
    d, n = X.shape

    def run(fn, mat, yy, coord_len, comp_len, tol, H, seed, timing=None):
        st = {}
        coord = torch.zeros(coord_len, dtype=torch.float64, device=dev)
        comp = torch.empty(comp_len, dtype=torch.float64, device=dev)
        kw = dict(timing=timing) if timing is not None else {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if fn == "primal":
            cabcd.primal_bcd(mat, yy, lam_of[fn], b_of[fn], s_of[fn], H, seed, w=coord, r=comp,
                             tol=tol, check_every=every, stats=st, **kw)
        else:
            cabcd.dual_bcd(mat, yy, lam_of[fn], b_of[fn], s_of[fn], H, seed, alpha=coord, w=comp,
                           tol=tol, check_every=every, stats=st, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st

    lam_of = {"primal": lam, "dual": 1e-5}
    b_of = {"primal": b, "dual": 16}
    s_of = {"primal": s, "dual": 8}
    zero = torch.zeros(d, dtype=torch.float64, device=dev)
    nrm0, _ = cabcd.primal_residual(X, lam, zero, -y)      # w = 0: r = -y
    tol = 0.1 * nrm0.item()
    H = 200000
    run("primal", X, y, d, n, tol, H, 2003)                  # warm-up
    el, st = run("primal", X, y, d, n, tol, H, 2003)
    tm = cabcd.new_timing()
    run("primal", X, y, d, n, tol, H, 2003, timing=tm)
    ph = cabcd.timing_dict(tm)["check"]
    rec["primal_resid_tol"] = {
        "tol_rel": 0.1, "check_every": every, "s": s, "b": b, "reached": st["h"] < H,
        "h": st["h"], "s_total": round(el, 4), "resid_rel": st["resid_norm"] / nrm0.item(),
        "check_ms": round(ph["ms"] / max(ph["launches"], 1), 4)}
    log(f"primal residual stop: {rec['primal_resid_tol']}")
    nA = A.shape[0]
    ynorm = float(torch.linalg.norm(yd))
    tol = 1e-2 * ynorm
    H = 80000
    run("dual", A, yd, nA, A.shape[1], tol, H, 2004)
    el, st = run("dual", A, yd, nA, A.shape[1], tol, H, 2004)
    tm = cabcd.new_timing()
    run("dual", A, yd, nA, A.shape[1], tol, H, 2004, timing=tm)
    ph = cabcd.timing_dict(tm)["check"]
    rec["sparse_dual_resid_tol"] = {
        "tol_rel": 1e-2, "check_every": every, "s": 8, "b": 16, "reached": st["h"] < H,
        "h": st["h"], "s_total": round(el, 4), "resid_rel": st["resid_norm"] / ynorm,
        "check_ms": round(ph["ms"] / max(ph["launches"], 1), 4)}
    log(f"sparse dual residual stop: {rec['sparse_dual_resid_tol']}")
    return rec


def time_to_tol(cabcd, torch, synth, tol=1e-6, d=4096, n=1 << 20, b=16, s=16, lam=1e-4,
                chunk=4, max_steps=400):
    log(f"time-to-{tol:g}: generating X ({d} x {n}) on the GPU")
    X, y, _, _ = synth.colscaled_ridge(d, n, 1003, device="cuda")
    torch.cuda.synchronize()
    res = {"workload": f"column-scaled dense primal, d={d} n={n} lambda={lam:g} b={b} s={s}, "
                       f"exact residual + objective every {chunk} outer steps",
           "tol": tol}

    def run(A, fstar):
        w = torch.zeros(d, dtype=torch.float64, device="cuda")
        r = torch.empty(n, dtype=torch.float64, device="cuda")
        trace = torch.zeros(1, dtype=torch.float64, device="cuda")
        # r_0 = X^T w_0 - y outside the timed region (a residual the caller holds)
        cabcd.primal_bcd(A, y, lam, b, s, 0, 7, w=w, r=r)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, err = 0, float("inf")
        while steps < max_steps:
            cabcd.primal_bcd(A, y, lam, b, s, chunk * s, 7, w=w, r=r, h0=steps * s,
                             flags=cabcd.FLAG_STATE_VALID, resid_every=chunk,
                             monitor_every=chunk, trace=trace)
            steps += chunk
            err = (trace.item() - fstar) / fstar
            if err <= tol:
                break
        return time.perf_counter() - t0, steps, err, w

    def gram_rate(A, elem, steps=32):
        """The Gram kernel alone over `steps` outer steps (HIP events around the
        Gram launches only): ms per launch, algorithmic bytes (the gathered
        rows) per second against the HBM peak, and flops per second.  Each
        event pair also holds the launch's dispatch (a few microseconds, a
        visible share of a 60 us launch)."""
        w = torch.zeros(d, dtype=torch.float64, device="cuda")
        r = torch.empty(n, dtype=torch.float64, device="cuda")
        tm = cabcd.new_timing()
        cabcd.primal_bcd(A, y, lam, b, s, steps * s, 11, w=w, r=r, timing=tm,
                         timing_mask=1 << cabcd.PHASES.index("gram"))
        g = cabcd.timing_dict(tm)["gram"]
        ms = g["ms"] / max(g["launches"], 1)
        sb = s * b
        gbs = sb * n * elem / (ms * 1e-3) / 1e9
        return {"gram_ms": round(ms, 4), "gram_gbs": round(gbs, 1),
                "hbm_frac": round(gbs / PEAK_HBM_GBS, 4),
                "gram_tflops": round(n * sb * (sb + 1) / (ms * 1e-3) / 1e12, 2)}

    # the optimum of the original FP64 X: the quantisation shift of each stored
    # problem is measured against it
    w_x, _ = closed_form(cabcd, torch, X, y, lam)
    for name, code in (("bf16", cabcd.BF16), ("fp8", cabcd.FP8_E4M3)):
        Q = cabcd.quantize(X, code)
        Xh = Q.dequantize()
        w_hat, fstar = closed_form(cabcd, torch, Xh, y, lam)
        shift = (torch.linalg.norm(w_hat - w_x) / torch.linalg.norm(w_x)).item()
        t64, st64, e64, w64 = run(Xh, fstar)
        g64 = gram_rate(Xh, 8)
        del Xh
        torch.cuda.empty_cache()
        tq, stq, eq, wq = run(Q, fstar)
        gq = gram_rate(Q, 2 if name == "bf16" else 1)
        nrm = torch.linalg.norm(w_hat)
        res[name] = {"fp64_on_xhat_s": round(t64, 5), "fp64_outer_steps": st64,
                     "fp64_rel_err": e64,
                     "mixed_s": round(tq, 5), "mixed_outer_steps": stq, "mixed_rel_err": eq,
                     "speedup": round(t64 / tq, 3), "gram_fp64": g64, "gram_" + name: gq,
                     # ||w^* - w*_X|| / ||w*_X||: how far storing X in this format
                     # moves the optimum (the problem the mixed runs solve is X^)
                     "quantisation_shift": shift,
                     # the final iterates against the optimum of X^, and the mixed
                     # iterate against the FP64 one (same blocks; equal only when
                     # both stopped after the same number of outer steps)
                     "fp64_w_rel_err": (torch.linalg.norm(w64 - w_hat) / nrm).item(),
                     "mixed_w_rel_err": (torch.linalg.norm(wq - w_hat) / nrm).item(),
                     "mixed_vs_fp64_w": (torch.linalg.norm(wq - w64) /
                                         torch.linalg.norm(w64)).item()}
        log(f"time-to-tol {name}: {res[name]}")
        del Q
        torch.cuda.empty_cache()
    return res


def batched_tol(cabcd, torch, synth, P=256, tol=1e-6, seed=1004, monitor=4, cheap=7,
                max_rounds=20000, baseline=True):
    """256 independent dense ridge problems (d, n, lambda log-uniform), time to a
    relative objective error of 1e-6 on every problem: the batched persistent
    path (one launch per round, hipGraph) against the one-problem path run
    problem after problem with the same (b, s), both on this GPU; FP64 and BF16
    storage (the BF16 runs solve the stored problem X^)."""
    ds, ns, lams = synth.ridge_batch(P, seed)
    log(f"batched: generating {P} problems (sum d*n = {sum(d * n for d, n in zip(ds, ns)):.3g})")
    data = [synth.gaussian_ridge(ds[p], ns[p], seed + 1 + p, device="cuda")[:2] for p in range(P)]
    # every X in the layout the library recommends (rows leading_dim apart:
    # 16-byte aligned, so the LDS-DMA Gram and 16-byte loads apply to all of
    # them, as they do to the quantised codes)
    data = [(padded(cabcd, X), y) for X, y in data]
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    def fstar(X, y, lam):
        return closed_form(cabcd, torch, X, y, lam)[1]

    res = {"workload": f"{P} Gaussian ridge problems, d log-uniform [32, 1024], n log-uniform "
                       f"[4096, 131072], lambda log-uniform [1e-6, 1e-1]; objective every "
                       f"{monitor} rounds (from the maintained residual, exact recomputation at "
                       f"every {cheap + 1}-th monitor point); stop at relative objective error "
                       f"{tol:g} on every problem",
           "problems": P, "sum_dn": int(sum(d * n for d, n in zip(ds, ns)))}
    for name in ("f64", "bf16"):
        if name == "f64":
            mats = [X for X, _ in data]
            fst = [fstar(X, y, lams[p]) for p, (X, y) in enumerate(data)]
        else:
            mats, fst = [], []
            for p, (X, y) in enumerate(data):
                Q = cabcd.quantize(X, cabcd.BF16)
                Xh = Q.dequantize()
                fst.append(fstar(Xh, y, lams[p]))
                del Xh
                mats.append(Q)
            torch.cuda.empty_cache()
        probs = [dict(X=mats[p], y=data[p][1], lam=lams[p], seed=2_000_000 + p,
                      f_target=fst[p] * (1 + tol)) for p in range(P)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B = cabcd.Batch(probs, monitor_every=monitor, cheap_monitors=cheap)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rounds, act = 0, P
        while act > 0 and rounds < max_rounds:
            act = B.run(monitor)
            rounds += monitor
        t2 = time.perf_counter()
        infos = [B.info(p) for p in range(P)]
        B.close()
        # the stopping test may use the maintained residual; check every problem
        # with an exact objective evaluation of its final w
        errs = [(cabcd.primal_objective(mats[p], data[p][1], lams[p], probs[p]["w"])[0].item()
                 - fst[p]) / fst[p] for p in range(P)]
        rec = {"plan_s": round(t1 - t0, 4), "solve_s": round(t2 - t1, 4), "rounds": rounds,
               "unconverged": act, "max_rel_err": max(errs),
               "ms_per_round": round((t2 - t1) / max(rounds, 1) * 1e3, 4)}
        pairs = {}
        for i in infos:
            k = f"b{i['b']}s{i['s']}"
            pairs[k] = pairs.get(k, 0) + 1
        rec["bs_choices"] = pairs
        # streamed bytes per problem: every outer step reads the gathered rows
        # twice (Gram, deferred update) plus r; an exact recomputation (a full
        # pass over X) at every (cheap + 1)-th monitor point
        e = 8 if name == "f64" else 2
        byts = 0.0
        for p, i in enumerate(infos):
            sb_p, n_p, st_p = i["b"] * i["s"], ns[p], i["steps"]
            exact = st_p // (monitor * (cheap + 1))
            byts += st_p * (2.0 * sb_p * n_p * e + 16.0 * n_p) + exact * (ds[p] * n_p * e + 16.0 * n_p)
        rec["stream_gb"] = round(byts / 1e9, 2)
        rec["hbm_gbs"] = round(byts / max(t2 - t1, 1e-9) / 1e9, 1)
        log(f"batched {name}: {rec}")
        if baseline:
            # one problem at a time, same storage, same (b, s), same stopping rule
            tot, steps_tot, worst = 0.0, 0, 0.0
            for p in range(P):
                X, y = mats[p], data[p][1]
                b, s = infos[p]["b"], infos[p]["s"]
                w = torch.zeros(ds[p], dtype=torch.float64, device="cuda")
                r = torch.empty(ns[p], dtype=torch.float64, device="cuda")
                tr = torch.zeros(1, dtype=torch.float64, device="cuda")
                cabcd.primal_bcd(X, y, lams[p], b, s, 0, 7, w=w, r=r)
                torch.cuda.synchronize()
                ta = time.perf_counter()
                steps, err = 0, float("inf")
                while steps < max_rounds:
                    # the same monitoring as the batch: f from the maintained r at
                    # `cheap` of every cheap+1 monitor points, exact at the others
                    exact = (steps // monitor + 1) % (cheap + 1) == 0
                    cabcd.primal_bcd(X, y, lams[p], b, s, monitor * s, 2_000_000 + p, w=w, r=r,
                                     h0=steps * s,
                                     flags=cabcd.FLAG_STATE_VALID | (
                                         0 if exact else cabcd.FLAG_MONITOR_MAINTAINED),
                                     resid_every=monitor if exact else 0,
                                     monitor_every=monitor, trace=tr)
                    steps += monitor
                    err = (tr.item() - fst[p]) / fst[p]
                    if err <= tol:
                        break
                tot += time.perf_counter() - ta
                steps_tot += steps
                worst = max(worst, err)
            rec["one_at_a_time_s"] = round(tot, 4)
            rec["one_at_a_time_outer_steps"] = steps_tot
            rec["one_at_a_time_max_rel_err"] = worst
            rec["speedup"] = round(tot / (t2 - t1), 3)
            log(f"one-at-a-time {name}: {tot:.3f} s, speedup {rec['speedup']}")
        res[name] = rec
        del probs, mats
        torch.cuda.empty_cache()
    return res


STAB_S = (1, 2, 4, 8, 16, 32)


def stability_curve(cabcd, torch, A, y, lam, b, s, H, points, seed, w_star, f_star,
                    dual=False):
    """One run of H iterations from zero, in `points` equal chunks (each a whole
    number of outer steps, so the iterates are those of one uninterrupted run);
    after every chunk the relative objective error of the primal iterate
    (f(w_h) - f*) / f* (objective recomputed from A) and its relative solution
    error ||w_h - w*|| / ||w*||, the two measures of the paper's stability
    study.  The dual reports its maintained w.  Returns [(h, obj, sol)]."""
    rows, cols = A.shape
    dev = y.device
    coord = torch.zeros(rows, dtype=torch.float64, device=dev)
    comp = torch.empty(cols, dtype=torch.float64, device=dev)
    run = cabcd.dual_bcd if dual else cabcd.primal_bcd
    kw = dict(alpha=coord, w=comp) if dual else dict(w=coord, r=comp)
    chunk = H // points
    assert chunk * points == H and chunk % s == 0
    run(A, y, lam, b, s, 0, seed, **kw)                # companion vector of the zero start
    nw = torch.linalg.norm(w_star)
    out = []
    for k in range(points):
        run(A, y, lam, b, s, chunk, seed, h0=k * chunk, flags=cabcd.FLAG_STATE_VALID, **kw)
        w = comp if dual else coord
        f = (cabcd.primal_objective_t(A, y, lam, w) if dual else
             cabcd.primal_objective(A, y, lam, w))[0].item()
        out.append(((k + 1) * chunk, (f - f_star) / f_star,
                    (torch.linalg.norm(w - w_star) / nw).item()))
    return out


def gram_conditions(cabcd, torch, A, scale, shift, b, s, seed, steps=16):
    """cond(G) of the s b x s b Gram and the largest cond(Gamma_j) of its b x b
    diagonal blocks (the matrices the solves factor) over the first `steps`
    outer steps of a run: medians and maxima."""
    import numpy as np
    idx = cabcd.sample(seed, 0, steps * s, b, A.shape[0]).reshape(steps, s * b)
    cg, cb = [], []
    for k in range(steps):
        G = cabcd.gram(A, idx[k].contiguous(), scale, shift)[0].cpu().numpy()
        cg.append(float(np.linalg.cond(G)))
        cb.append(max(float(np.linalg.cond(G[j * b:(j + 1) * b, j * b:(j + 1) * b]))
                      for j in range(s)))
    return {"G_median": float(np.median(cg)), "G_max": max(cg),
            "block_median": float(np.median(cb)), "block_max": max(cb)}


def stability(cabcd, torch, synth, seed=2005, points=32):
    """Numerical stability of the s-step methods (Section 6, the CA-BCD and
    CA-BDCD convergence figures) on synthetic stand-ins with the paper's
    regularisation rule, lambda = 1000 x the smallest eigenvalue of X X^T / n:
    relative objective and solution error against iterations for
    s = 1 ... 32 with one block sequence, run until FP64 reaches its floor;
    FP64 and the BF16 / FP8 storage (each against the optimum of its own
    stored matrix); and the condition numbers of the Gram matrices per s.
    Primal: X = U diag(sigma) V^T, d = 512, n = 32768, sigma 1..1e3, b = 16,
    H = 65536.  Dual: the same construction with d = 256, n = 1024, b' = 16,
    H' = 32768 (A = X^T)."""
    dev = "cuda"
    res = {"s": list(STAB_S), "points": points,
           "lambda_rule": "1000 x the smallest eigenvalue of X X^T / n (sigma_min = 1)"}
    cases = {
        "primal": dict(d=512, n=32768, b=16, H=65536, dual=False, data_seed=1010),
        "dual": dict(d=256, n=1024, b=16, H=32768, dual=True, data_seed=1011),
    }
    for meth, c in cases.items():
        d, n, b, H, dual = c["d"], c["n"], c["b"], c["H"], c["dual"]
        X, y, _ = synth.spectral_ridge(d, n, c["data_seed"], sigma_max=1e3, device=dev)
        lam = 1000.0 / n
        rec = {"workload": f"X = U diag(sigma) V^T, d={d}, n={n}, sigma 1..1e3, "
                           f"lambda={lam:.4g}, b={b}, H={H}, from zero",
               "lambda": lam, "b": b, "H": H}
        for fmt in ("f64", "bf16", "fp8"):
            if fmt == "f64":
                Xs = X
                store = X.t().contiguous() if dual else X
            else:
                code = cabcd.BF16 if fmt == "bf16" else cabcd.FP8_E4M3
                store = cabcd.quantize(X.t().contiguous() if dual else X, code)
                Xs = store.dequantize()
                Xs = Xs.t().contiguous() if dual else Xs
            w_star, f_star = closed_form(cabcd, torch, Xs, y, lam)
            curves = {}
            t0 = time.perf_counter()
            for s_ in STAB_S:
                pts = stability_curve(cabcd, torch, store, y, lam, b, s_, H, points, seed,
                                      w_star, f_star, dual=dual)
                curves[f"s{s_}"] = {"h": [p[0] for p in pts], "obj": [p[1] for p in pts],
                                    "sol": [p[2] for p in pts]}
            s1 = curves["s1"]
            keep = list(range(points // 8 - 1, points, points // 8))   # 8 points a curve

            def thin(v):
                return [float(f"{v[i]:.3g}") for i in keep]
            rec[fmt] = {
                "h": [curves["s1"]["h"][i] for i in keep],
                "obj": {k: thin(v["obj"]) for k, v in curves.items()},
                "sol": {k: thin(v["sol"]) for k, v in curves.items()},
                # the largest gap of each s to s = 1 over all monitor points
                "max_sol_gap_vs_s1": {k: float(f"{max(abs(a - b_) for a, b_ in zip(v['sol'], s1['sol'])):.3g}")
                                      for k, v in curves.items()},
                "seconds": round(time.perf_counter() - t0, 3)}
            log(f"stability {meth} {fmt}: sol {rec[fmt]['sol']}")
            del store, Xs
        A = X.t().contiguous() if dual else X
        scale, shift = (1.0 / (lam * n * n), 1.0 / n) if dual else (1.0 / n, lam)
        rec["cond"] = {f"s{s_}": gram_conditions(cabcd, torch, A, scale, shift, b, s_, seed)
                       for s_ in STAB_S}
        log(f"stability {meth} cond: {rec['cond']}")
        res[meth] = rec
        del X, y, A
        torch.cuda.empty_cache()
    return res


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
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 1 GiB three times")
        return
    cabcd.load()
    if args.only_batch:
        print(json.dumps({"batched_tol": batched_tol(cabcd, torch, synth,
                                                     baseline=not args.batch_no_baseline)}),
              flush=True)
        return
    if args.only_tol:
        print(json.dumps({"time_to_tol": time_to_tol(cabcd, torch, synth)}), flush=True)
        return
    if args.only_extra:
        log(f"generating X ({args.d} x {args.n}, FP64) on the GPU")
        X, y, _ = synth.spectral_ridge(args.d, args.n, 1001, device="cuda:0")
        X = padded(cabcd, X)
        torch.cuda.synchronize()
        print(json.dumps({"extra": extra_records(args, cabcd, torch, synth, X, y)}), flush=True)
        return
    if args.only_sparse:
        print(json.dumps({"sparse": sparse_records(cabcd, torch, synth)[0]}), flush=True)
        return
    if args.only_stability:
        print(json.dumps({"stability": stability(cabcd, torch, synth)}), flush=True)
        return
    out, X, y = headline(args, cabcd, torch, synth)
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(X, y, args.lam, args.b, args.s, args.cpu_steps, 2001)
    else:
        out["cpu_baseline"] = None
    if not args.no_extra:
        out["extra"] = extra_records(args, cabcd, torch, synth, X, y)
    del X, y
    torch.cuda.empty_cache()
    if not args.no_stability:
        out["stability"] = stability(cabcd, torch, synth)
    if not args.no_tol:
        out["time_to_tol"] = time_to_tol(cabcd, torch, synth)
    if not args.no_batch:
        out["batched_tol"] = batched_tol(cabcd, torch, synth)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
