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
on.  cpu_baseline: the FP64 oracle on a bounded number of outer steps of the
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
    ap.add_argument("--cpu-steps", type=int, default=4)
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
    ap.add_argument("--only-stability", action="store_true",
                    help="run only the headline and the numerical-stability record")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM bytes per Gram launch measured by rocprofv3 counters")
    return ap.parse_args()


def cpu_baseline(X, y, lam, b, s, steps, seed):
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
    per_step = (stamps[-1] - t0) / steps
    flops = n * sb * (sb + 1)
    return {"value": flops / per_step / 1e12, "unit": "TFLOP/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{steps} outer steps (s={s}, b={b}) of the FP64 oracle on the same "
                      f"d={d} x n={n} problem; {per_step:.3f} s per step"}


def timed_primal(cabcd, torch, X, y, lam, b, s, steps, warmup, seed, dual=False, mask=0):
    """Warm up, then time `steps` outer steps; returns (elapsed s, phase dict).
    `mask` selects the phases bracketed by HIP events (0: all); every event
    pair costs GPU time, so the timed headline run brackets the Gram only."""
    rows, cols = X.shape
    coord = torch.zeros(rows, dtype=torch.float64, device=y.device)
    comp = torch.empty(cols, dtype=torch.float64, device=y.device)
    run = cabcd.dual_bcd if dual else cabcd.primal_bcd
    if dual:
        kw0 = dict(alpha=coord, w=comp)
    else:
        kw0 = dict(w=coord, r=comp)
    run(X, y, lam, b, s, warmup * s, seed, **kw0)
    torch.cuda.synchronize()
    tm = cabcd.new_timing()
    t0 = time.perf_counter()
    run(X, y, lam, b, s, steps * s, seed, h0=warmup * s, flags=cabcd.FLAG_STATE_VALID,
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


def headline(args, cabcd, torch, synth):
    dev = "cuda:0"
    d, n, b, s, lam = args.d, args.n, args.b, args.s, args.lam
    sb = s * b
    log(f"generating X ({d} x {n}, FP64) on the GPU")
    X, y, _ = synth.spectral_ridge(d, n, 1001, device=dev)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    gram_only = 1 << cabcd.PHASES.index("gram")
    elapsed, ph = timed_primal(cabcd, torch, X, y, lam, b, s, args.steps, args.warmup, 2001,
                               mask=gram_only)
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
    return out, X, y


def extra_records(args, cabcd, torch, synth, X, y):
    """Other shapes of the path (events bracket the Gram only, so the step
    times carry no timing overhead); per_iteration_us = step time / s, the cost
    of one b-coordinate iteration, shows what the s-step form saves."""
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
    el, ph = timed_primal(cabcd, torch, XT, y, lam, args.b, args.s, 20, 2, 2001, dual=True,
                          mask=gram_only)
    g = ph["gram"]["ms"] / 20
    sb = args.s * args.b
    rec["dual_s32"] = {"ms_per_step": round(el / 20 * 1e3, 4), "gram_ms": round(g, 4),
                       "gram_tflops": round(d * sb * (sb + 1) / (g * 1e-3) / 1e12, 3)}
    log(f"dual: {rec['dual_s32']}")
    del XT
    # sparse dual: A = X^T in CSR, 20000 rows x 2^20 columns, 315 Zipf(1.1) features per row
    import numpy as np
    log("generating the sparse problem (CSR, 20000 x 2^20)")
    rowptr, colidx, vals, ys, _ = synth.zipf_csr_ridge(20000, 1 << 20, 315, 1002)
    A = cabcd.CSR(torch.tensor(rowptr, device="cuda"), torch.tensor(colidx, device="cuda"),
                  torch.tensor(vals, device="cuda"), (20000, 1 << 20))
    yd = torch.tensor(ys, device="cuda")
    for s in (1, 8, 32):
        b = 16
        el, ph = timed_primal(cabcd, torch, A, yd, 1e-5, b, s, 20, 2, 2002, dual=True,
                              mask=gram_only)
        # per outer step: the Grams of several future steps come from one launch,
        # the Y u of each step from its own
        g = ph["gram"]["ms"] / 20
        # algorithmic Gram work of the sampled rows: 2 sum_c nnz_c(I)^2 flops over the
        # nnz of the gathered rows (12 bytes each), averaged over the timed steps
        idx = cabcd.sample(2002, 2 * s, 20 * s, b, 20000).cpu().numpy().reshape(20, s * b)
        fl, by = [], []
        for blk in idx:
            cols = np.concatenate([colidx[rowptr[i]:rowptr[i + 1]] for i in blk])
            cnt = np.bincount(cols)
            fl.append(2.0 * float((cnt.astype(np.float64) ** 2).sum()))
            by.append(12.0 * len(cols))
        rec[f"sparse_dual_s{s}"] = {
            "ms_per_step": round(el / 20 * 1e3, 4), "gram_ms": round(g, 4),
            "gram_gflops": round(np.mean(fl) / (g * 1e-3) / 1e9, 2),
            "gram_gbs": round(np.mean(by) / (g * 1e-3) / 1e9, 2)}
        log(f"sparse dual s={s}: {rec[f'sparse_dual_s{s}']}")
    rec.update(resid_tol_records(cabcd, torch, X, y, lam, args.b, args.s, A, yd))
    return rec


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

    def closed_form_fstar(Xh):
        M = Xh @ Xh.t()
        M /= n
        M.diagonal().add_(lam)
        L = torch.linalg.cholesky(M)
        rhs = (Xh @ y) / n
        w = torch.cholesky_solve(rhs[:, None], L)[:, 0]
        del M, L
        f, _ = cabcd.primal_objective(Xh, y, lam, w)
        return f.item()

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
        return time.perf_counter() - t0, steps, err

    def gram_rate(A, elem, steps=8):
        """The Gram kernel alone over `steps` outer steps (HIP events around the
        Gram launches only): ms per launch, algorithmic bytes (the gathered
        rows) per second against the HBM peak, and flops per second."""
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

    for name, code in (("bf16", cabcd.BF16), ("fp8", cabcd.FP8_E4M3)):
        Q = cabcd.quantize(X, code)
        Xh = Q.dequantize()
        fstar = closed_form_fstar(Xh)
        t64, st64, e64 = run(Xh, fstar)
        g64 = gram_rate(Xh, 8)
        del Xh
        torch.cuda.empty_cache()
        tq, stq, eq = run(Q, fstar)
        gq = gram_rate(Q, 2 if name == "bf16" else 1)
        res[name] = {"fp64_on_xhat_s": round(t64, 5), "fp64_outer_steps": st64,
                     "fp64_rel_err": e64,
                     "mixed_s": round(tq, 5), "mixed_outer_steps": stq, "mixed_rel_err": eq,
                     "speedup": round(t64 / tq, 3), "gram_fp64": g64, "gram_" + name: gq}
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
    torch.cuda.synchronize()

    def fstar(X, y, lam):
        n = X.shape[1]
        M = X @ X.t()
        M /= n
        M.diagonal().add_(lam)
        L = torch.linalg.cholesky(M)
        w = torch.cholesky_solve(((X @ y) / n)[:, None], L)[:, 0]
        f, _ = cabcd.primal_objective(X, y, lam, w)
        return f.item()

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
        if name == "f64" and baseline:
            # one problem at a time, same (b, s), same stopping rule
            tot, steps_tot, worst = 0.0, 0, 0.0
            for p in range(P):
                X, y = data[p]
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
            log(f"one-at-a-time f64: {tot:.3f} s, speedup {rec['speedup']}")
        res[name] = rec
        del probs, mats
        torch.cuda.empty_cache()
    return res


def stability(cabcd, torch, X, y, lam, b=8, H=4096, seed=2005):
    """Numerical stability (Section 6) on the synthetic stand-in: the same
    block sequence run with s = 1 ... 32 must give the same iterates up to
    rounding (CA-BCD reproduces BCD in exact arithmetic), in FP64 and on BF16
    storage; and the condition numbers of the s-step Gram G and of its b x b
    diagonal blocks (the matrices actually factorised) over sampled outer
    steps, for the primal (rows of X) and the dual (columns of X)."""
    import numpy as np
    d, n = X.shape
    log("stability: closed-form optimum")
    M = X @ X.T
    M /= n
    M.diagonal().add_(lam)
    L = torch.linalg.cholesky(M)
    wst = torch.cholesky_solve(((X @ y) / n)[:, None], L)[:, 0]
    del M, L
    fst = cabcd.primal_objective(X, y, lam, wst)[0].item()
    res = {"workload": f"the headline matrix (d={d}, n={n}, spectrum 1..1e3, lambda={lam:g}), "
                       f"b={b}, H={H} iterations from w=0 with one block sequence",
           "H": H, "b": b}
    for name in ("f64", "bf16"):
        A, fs = X, fst
        if name == "bf16":
            A = cabcd.quantize(X, cabcd.BF16)
            Xh = A.dequantize()
            M = Xh @ Xh.T
            M /= n
            M.diagonal().add_(lam)
            L = torch.linalg.cholesky(M)
            wh = torch.cholesky_solve(((Xh @ y) / n)[:, None], L)[:, 0]
            fs = cabcd.primal_objective(Xh, y, lam, wh)[0].item()
            del Xh, M, L, wh
        rec, w1 = {}, None
        for s_ in (1, 2, 4, 8, 16, 32):
            w, _ = cabcd.primal_bcd(A, y, lam, b, s_, H, seed)
            f = cabcd.primal_objective(A, y, lam, w)[0].item()
            if w1 is None:
                w1 = w.clone()
            rec[f"s{s_}"] = {"rel_obj_err": (f - fs) / fs,
                             "w_rel_diff_vs_s1": (torch.linalg.norm(w - w1) /
                                                  torch.linalg.norm(w1)).item()}
        res[name] = rec
        log(f"stability {name}: {rec}")
        del A
    torch.cuda.empty_cache()

    def conds(gram_of_step, steps, s_, bb):
        cg, cb = [], []
        for k in range(steps):
            G = gram_of_step(k).cpu().numpy()
            cg.append(float(np.linalg.cond(G)))
            cb.append(max(float(np.linalg.cond(G[j * bb:(j + 1) * bb, j * bb:(j + 1) * bb]))
                          for j in range(s_)))
        return {"G_median": float(np.median(cg)), "G_max": max(cg),
                "diag_block_median": float(np.median(cb)), "diag_block_max": max(cb)}

    cond = {}
    for s_ in (8, 32):
        idx = cabcd.sample(seed, 0, 16 * s_, b, d).reshape(16, s_ * b)
        cond[f"primal_s{s_}"] = conds(
            lambda k: cabcd.gram(X, idx[k].contiguous(), 1.0 / n, lam)[0], 16, s_, b)
        jdx = cabcd.sample(seed, 0, 16 * s_, b, n).reshape(16, s_ * b).long()
        ar = torch.arange(s_ * b, dtype=torch.int32, device=X.device)

        def dual_gram(k):
            Y = X[:, jdx[k]].t().contiguous()   # the sampled data points (rows of X^T)
            return cabcd.gram(Y, ar, 1.0 / (lam * n * n), 1.0 / n)[0]
        cond[f"dual_s{s_}"] = conds(dual_gram, 16, s_, b)
    res["cond"] = cond
    log(f"stability cond: {cond}")
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
        torch.cuda.synchronize()
        print(json.dumps({"extra": extra_records(args, cabcd, torch, synth, X, y)}), flush=True)
        return
    out, X, y = headline(args, cabcd, torch, synth)
    if args.only_stability:
        print(json.dumps({"stability": stability(cabcd, torch, X, y, args.lam)}), flush=True)
        return
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(X, y, args.lam, args.b, args.s, args.cpu_steps, 2001)
    else:
        out["cpu_baseline"] = None
    if not args.no_extra:
        out["extra"] = extra_records(args, cabcd, torch, synth, X, y)
    if not args.no_stability:
        out["stability"] = stability(cabcd, torch, X, y, args.lam)
    del X, y
    torch.cuda.empty_cache()
    if not args.no_tol:
        out["time_to_tol"] = time_to_tol(cabcd, torch, synth)
    if not args.no_batch:
        out["batched_tol"] = batched_tol(cabcd, torch, synth)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
