#!/usr/bin/env python3
"""Benchmark: S_k(A) time and GEMM TFLOP/s on one MI355X.

Default workload (one step = one evaluation of S_k(A)):
    large_symmetric: n = 4096, k = 729 = 9^3, A = Q diag(lam) Q^T with
    lam ~ U[-0.95, 0.95], seed 2; radix-9 (15 products) in FP64.
In the same run, with the same protocol: binary splitting (20 products,
k_eff = 1024) in FP64, and both methods in FP32.

`value` is logical GEMM TFLOP/s of the radix-9 FP64 step: (products x 2 n^3)
/ step time, inputs resident in HBM before the timed region.  The JSON line
also carries the per-launch roofline of the FP64 product kernel (HIP events
around every product launch on the call's stream during the timed steps) and
the CPU oracle timed on the host's cores.

Other workloads (`--workload`): gaussian_rho (n = 8192 FP32, k = 3375,
radix-15 vs radix-9 vs binary), precision_sym (n = 8192, k = 729, mixed
precision forms), jacobi_batch (2048 small matrices, persistent batched
launch vs per-matrix loop).  Each prints its own JSON line.
"""

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

METRIC = "S_k(A) time + GEMM TFLOP/s (%MFMA peak), radix-9/15 vs squaring at stated err"
PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2516.6, "f16": 2516.6}   # dense TFLOP/s, MI355X
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large_symmetric",
                    choices=["large_symmetric", "gaussian_rho", "precision_sym", "jacobi_batch",
                             "small_symmetric", "all"])
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip timing the CPU oracle (profiling runs)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    ap.add_argument("--only", default="",
                    help="comma list of method:dtype legs to run (profiling runs)")
    return ap.parse_args()


def time_leg(ns, h, A, k, method, dtype, out, steps, warmup, stream, n, separate_events=False):
    """Time `steps` evaluations after `warmup`; per-product HIP-event timing
    on the call's stream during the timed steps.  separate_events: the timed
    steps run without the events (at small n the event records between
    launches are a large part of a call), and a second pass of as many steps
    records them for the per-launch figures."""
    import torch
    k_eff, levels, products = ns.ns_plan(k, method)
    fn = lambda: ns.ns_eval_ex(A, k, method, dtype, out=out, handle=h, stream=stream)  # noqa: E731
    log(f"[bench] {method} {dtype} n={n} k={k}: warmup {warmup}, steps {steps}")
    fn()                                            # workspace allocation
    torch.cuda.synchronize()
    h.ns_set_product_timing(not separate_events)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    h.ns_product_timing(reset=True)                 # keep only the timed steps' launches
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    if separate_events:
        h.ns_set_product_timing(True)
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
    cnt, kms, kfl = h.ns_product_timing(reset=True)
    h.ns_set_product_timing(False)
    flops = products * 2.0 * n ** 3
    peak = PEAK["f64" if dtype == "f64" else ("bf16" if dtype in ("split_bf16", "f16_scaled") else "f32")]
    r = {"ms": sec * 1e3, "tflops": flops / sec / 1e12, "products": products, "k_eff": k_eff,
         "pct_peak_of_dtype": 100.0 * flops / sec / 1e12 / peak,
         "product_launches": cnt, "product_avg_ms": kms / max(cnt, 1),
         "product_tflops": kfl / (kms * 1e-3) / 1e12 if kms > 0 else None}
    log(f"[bench]   {sec * 1e3:.2f} ms/step  {flops / sec / 1e12:.2f} TFLOP/s  "
        f"product avg {kms / max(cnt, 1):.3f} ms")
    return r


def rnd(d):
    return {k: (round(v, 6) if isinstance(v, float) else v) for k, v in d.items()}


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        info = [p for p in threadpool_info() if p.get("internal_api") in ("openblas", "mkl", "blis")]
        if info:
            return int(info[0]["num_threads"])
    except Exception:
        pass
    return os.cpu_count()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def sampled_cols(n, count, seed=0):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, count, replace=False))


def cpu_oracle_sample(fn, label, flops, min_seconds=10.0, max_runs=50):
    """Time the oracle (test/benchmark infrastructure) on a bounded sample:
    `fn` (worth `flops`) is run until at least min_seconds have passed (at
    most max_runs times); the rate is the mean over the runs, and the first
    run's result is returned."""
    thr = blas_threads()
    log(f"[bench] cpu oracle: {label} on {thr} threads")
    t0 = time.perf_counter()
    res = fn()
    runs = 1
    while time.perf_counter() - t0 < min_seconds and runs < max_runs:
        fn()
        runs += 1
    total = time.perf_counter() - t0
    sec = total / runs
    log(f"[bench]   cpu {runs} run(s), {sec:.2f} s each")
    return res, {"value": round(flops / sec / 1e12, 4), "unit": "TFLOP/s", "cores": thr,
                 "kind": "oracle",
                 "sample": f"{label}: {runs} run(s), {sec:.2f} s each, {total:.1f} s in all ({cpu_model()})"}


def measured_traffic(summary="pmc_product_f64_large_symmetric.md", root=None):
    """HBM-side bytes per launch of the FP64 product kernel from the committed
    rocprofv3 counter summary, or None once the kernel source or the product
    schedule (which sets each launch's epilogue) has changed since the
    counters were taken (the summary records a source hash)."""
    import hashlib
    root = root or os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", summary)
    try:
        vals = {}
        with open(path) as fh:
            for line in fh:
                parts = line.split()
                if len(parts) == 2 and parts[0] in ("source_sha256_16", "traffic_bytes_per_launch"):
                    vals[parts[0]] = parts[1]
        h = hashlib.sha256()
        for f in ("gemm_device.h", "gemm.hip", "ns.cpp"):
            with open(os.path.join(root, "paper_2602_11843_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
        if vals.get("source_sha256_16") != h.hexdigest()[:16]:
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def roofline_from_leg(leg, n, kernel, dtype, mfma_per_logical=1.0):
    if not leg.get("product_launches"):
        return None
    peak = PEAK[dtype]
    achieved = mfma_per_logical * 2.0 * n ** 3 / (leg["product_avg_ms"] * 1e-3) / 1e12
    return {"bound": "mfma", "kernel": kernel, "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
            "per_launch_flops": mfma_per_logical * 2.0 * n ** 3,
            "avg_launch_ms": round(leg["product_avg_ms"], 5), "launches": leg["product_launches"]}


def base_line(args, value, ms, dtype, config):
    return {"metric": METRIC, "value": round(value, 4), "unit": "TFLOP/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


def select(legs, args):
    if not args.only:
        return legs
    want = [tuple(x.split(":")) for x in args.only.split(",")]
    return [l for l in legs if l in want]


def bench_large_symmetric(args, torch, ns):
    """n = 4096, k = 729: radix-9 vs binary in FP64 and FP32 (the headline)."""
    import workloads
    from oracle import series                      # benchmark infrastructure only
    w = workloads.make("large_symmetric")
    n, k = w.A.shape[0], 729
    h = ns.Handle(0)
    stream = torch.cuda.current_stream()
    A64 = torch.from_numpy(w.A).cuda()
    A32 = A64.float()
    out64, out32 = torch.empty_like(A64), torch.empty_like(A32)
    legs = select([("radix9", "f64"), ("binary", "f64"), ("radix9", "f32"), ("binary", "f32")], args)
    res, errs = {}, {}
    cols = sampled_cols(n, 64)
    for method, dtype in legs:
        A, out = (A64, out64) if dtype == "f64" else (A32, out32)
        res[(method, dtype)] = time_leg(ns, h, A, k, method, dtype, out, args.steps, args.warmup,
                                        stream, n)
        got = out.double().cpu().numpy()
        ref = series.spectral_form(w.Q, w.lam, res[(method, dtype)]["k_eff"], cols=cols)
        errs[(method, dtype)] = series.rel_fro(got[:, cols], ref)
    key = ("radix9", "f64") if ("radix9", "f64") in res else next(iter(res))
    main = res[key]
    cpu, err_full = None, None
    if not args.no_cpu_baseline:
        S_cpu, cpu = cpu_oracle_sample(lambda: series.radix9(w.A, k)[0],
                                       "whole workload once: radix-9 S_729(A), n=4096, 15 float64 products",
                                       15 * 2.0 * n ** 3)
        if ("radix9", "f64") in res:
            ns.ns_eval_ex(A64, k, "radix9", "f64", out=out64, handle=h, stream=stream)
            torch.cuda.synchronize()
            err_full = series.rel_fro(out64.cpu().numpy(), S_cpu)
    line = base_line(args, main["tflops"], main["ms"], key[1],
                     {"workload": "large_symmetric", "n": n, "k": k, "method": key[0],
                      "k_eff": main["k_eff"], "products": main["products"], "seed": w.seed,
                      "lam": "U[-0.95,0.95]"})
    line["pct_mfma_peak"] = round(100.0 * main["tflops"] / PEAK[key[1]], 2)
    line["rel_err_vs_definition_sampled"] = errs[key]
    line["rel_err_vs_cpu_oracle"] = err_full
    line["legs"] = {f"{m}:{d}": {**rnd(r), "rel_err_sampled": errs[(m, d)]} for (m, d), r in res.items()}
    for d in ("f64", "f32"):
        if ("radix9", d) in res and ("binary", d) in res:
            line[f"radix9_over_binary_speedup_{d}"] = round(res[("binary", d)]["ms"] / res[("radix9", d)]["ms"], 4)
    line["predicted_speedup_by_product_count"] = round(20 / 15, 4)
    kern = "gemm_kernel<PolF64M16<2,2,4,4>>" if key[1] == "f64" else "gemm_kernel<PolF32<2,2,4,8>>"
    line["roofline"] = roofline_from_leg(main, n, kern, key[1])
    if line["roofline"] and key == ("radix9", "f64"):
        line["roofline"]["traffic"] = measured_traffic()
        line["roofline"]["traffic_unit"] = "bytes per launch (FETCH_SIZE x2 + WRITE_SIZE, copy-calibrated)"
    line["cpu_baseline"] = cpu
    return line


def bench_gaussian_rho(args, torch, ns):
    """n = 8192 FP32, nonsymmetric N(0,1)/sqrt(n) scaled to rho_hat = 0.99,
    k = 3375: radix-15 with the contraction-aware table (18 products, the
    reported value) and with the App. B table (18, diverges here) vs radix-9
    (20, k_eff 6561) vs binary (24, k_eff 4096) vs the exact any-k plan (19,
    k itself), with per-level norms; plus the same matrix rescaled to
    rho_hat = 0.95, inside the App. B kernel's convergence domain."""
    import scipy.linalg
    import workloads
    from oracle import series
    log("[bench] generating gaussian_rho input (n=8192, 400 power iterations)")
    g = workloads.make("gaussian_rho")
    n, k = g.A.shape[0], 3375
    h = ns.Handle(0)
    stream = torch.cuda.current_stream()
    cols = sampled_cols(n, 16)
    I_cols = np.zeros((n, len(cols)))
    I_cols[cols, np.arange(len(cols))] = 1.0
    out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    res, errs, norms = {}, {}, {}
    for rho in (0.99, 0.95):
        A = g.A * (rho / 0.99)
        log(f"[bench] LU reference (I - A)^-1 e_j for rho {rho}")
        lu = scipy.linalg.lu_factor(np.eye(n) - A)
        ref = scipy.linalg.lu_solve(lu, I_cols)          # S_inf columns; A^k is negligible
        del lu
        Ad = torch.from_numpy(A).float().cuda()
        legs = ([("radix15c", "f32"), ("radix15", "f32"), ("radix9", "f32"), ("binary", "f32"),
                 ("mixed", "f32")] if rho == 0.99 else [("radix15", "f32")])
        for method, dtype in select(legs, args):
            key = (method, dtype, rho)
            res[key] = time_leg(ns, h, Ad, k, method, dtype, out, args.steps, args.warmup, stream, n)
            _, rep = ns.ns_eval_ex(Ad, k, method, dtype, out=out, handle=h, stream=stream, report=True)
            got = out.double().cpu().numpy()
            errs[key] = series.rel_fro(got[:, cols], ref)
            norms[key] = rep["level_norm"]
            log(f"[bench]   rho {rho} {method}: sampled rel err vs (I-A)^-1 {errs[key]:.3e}, "
                f"level norms {['%.3g' % x for x in rep['level_norm']]}")
        del Ad
    key = ("radix15c", "f32", 0.99) if ("radix15c", "f32", 0.99) in res else next(iter(res))
    main = res[key]
    cpu = None
    if not args.no_cpu_baseline:
        # bounded sample: one radix-15 level of the oracle (6 float64 products at n = 8192)
        _, cpu = cpu_oracle_sample(lambda: series.radix15(g.A, 15),
                                   "one radix-15 level of the oracle at n=8192 (6 float64 products)",
                                   6 * 2.0 * n ** 3)
    line = base_line(args, main["tflops"], main["ms"], "f32",
                     {"workload": "gaussian_rho", "n": n, "k": k, "method": key[0], "rho_hat": 0.99,
                      "k_eff": main["k_eff"], "products": main["products"], "seed": g.seed})
    line["legs"] = {f"{m}:{d}:rho{r}": {**rnd(v), "rel_err_sampled_vs_inverse": errs[(m, d, r)],
                                        "level_norm": norms[(m, d, r)]}
                    for (m, d, r), v in res.items()}
    if ("binary", "f32", 0.99) in res:
        b = res[("binary", "f32", 0.99)]["ms"]
        line["speedup_over_binary"] = {m: round(b / res[(m, "f32", 0.99)]["ms"], 4)
                                       for m in ("radix15c", "radix15", "radix9", "mixed") if (m, "f32", 0.99) in res}
        line["predicted_speedup_by_product_count"] = {"radix15c": round(24 / 18, 4),
                                                      "radix15": round(24 / 18, 4), "radix9": round(24 / 20, 4),
                                                      "mixed": round(24 / series.plan(k, "mixed")[2], 4)}
    line["roofline"] = roofline_from_leg(main, n, "gemm_kernel<PolF32<2,2,4,8>>", "f32")
    line["cpu_baseline"] = cpu
    return line


def bench_precision_sym(args, torch, ns):
    """n = 8192, k = 729, symmetric lam ~ U[-0.9, 0.9]: radix-9 with the
    products in FP64, FP32, FP32 + FP64 accumulation, split-BF16 and scaled
    FP16, in the telescoping form and in the residual form (FP64 residual)."""
    import workloads
    from oracle import series
    log("[bench] generating precision_sym input (n=8192)")
    w = workloads.make("precision_sym")
    n, k = w.A.shape[0], 729
    h = ns.Handle(0)
    stream = torch.cuda.current_stream()
    A64 = torch.from_numpy(w.A).cuda()
    A32 = A64.float()
    out64, out32 = torch.empty_like(A64), torch.empty_like(A32)
    cols = sampled_cols(n, 32)
    legs = select([("radix9", "split_bf16"), ("radix9", "f16_scaled"), ("radix9", "f32_acc64"),
                   ("radix9", "f32"), ("radix9", "f64"), ("radix9_resid", "split_bf16"),
                   ("radix9_resid", "f16_scaled"), ("radix9_resid", "f32_acc64")], args)
    res, errs = {}, {}
    for method, dtype in legs:
        A, out = (A32, out32) if dtype == "f32" else (A64, out64)
        res[(method, dtype)] = time_leg(ns, h, A, k, method, dtype, out, args.steps, args.warmup, stream, n)
        got = out.double().cpu().numpy()
        ref = series.spectral_form(w.Q, w.lam, res[(method, dtype)]["k_eff"], cols=cols)
        errs[(method, dtype)] = series.rel_fro(got[:, cols], ref)
        log(f"[bench]   rel err vs FP64 definition (sampled) {errs[(method, dtype)]:.3e}")
    key = ("radix9", "split_bf16") if ("radix9", "split_bf16") in res else next(iter(res))
    main = res[key]
    cpu = None
    if not args.no_cpu_baseline:
        _, cpu = cpu_oracle_sample(lambda: series.radix9(w.A, 9),
                                   "one radix-9 level of the oracle at n=8192 (5 float64 products)",
                                   5 * 2.0 * n ** 3)
    line = base_line(args, main["tflops"], main["ms"], "bf16x3+f64",
                     {"workload": "precision_sym", "n": n, "k": k, "method": key[0],
                      "precision": key[1], "k_eff": main["k_eff"], "products": main["products"],
                      "seed": w.seed, "lam": "U[-0.9,0.9]"})
    line["legs"] = {f"{m}:{d}": {**rnd(r), "rel_err_vs_fp64_definition_sampled": errs[(m, d)]}
                    for (m, d), r in res.items()}
    line["roofline"] = roofline_from_leg(main, n, "gemm_panel_kernel<PolPanel<2,4,4,2,true,1,2,2>>", "bf16",
                                         mfma_per_logical=3.0)
    line["cpu_baseline"] = cpu
    return line


def bench_jacobi_batch(args, torch, ns):
    """2048 FP32 Jacobi matrices, n uniform on {8,...,256}, k = 81 radix-9:
    one persistent launch replayed from a cached HIP graph (tiles autotuned)
    against the per-matrix launch loop."""
    import workloads
    from oracle import series
    w = workloads.make("jacobi_batch")
    buf, offs = w.packed(np.float32)
    A = torch.from_numpy(buf).cuda()
    offd = torch.from_numpy(offs).cuda()
    nh = torch.from_numpy(w.ns.astype(np.int32))
    nd = nh.cuda()
    out = torch.empty_like(A)
    k = 81
    flops = float(sum(10 * 2.0 * int(m) ** 3 for m in w.ns))
    h = ns.Handle(0)
    # the autotuner's pick is also written to this JSON-lines file
    os.environ.setdefault("NS_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "ns_tune.jsonl"))
    os.makedirs(os.path.dirname(os.environ["NS_TUNE_CACHE"]) or ".", exist_ok=True)
    log("[bench] autotuning the batched kernel")
    timed = ns.ns_autotune_batched(A, offd, nd, nh, k, out, handle=h)
    log(f"[bench]   {timed} configurations timed")
    fn = lambda: ns.ns_eval_batched(A, offd, nd, nh, k, "radix9", "f32", out_packed=out, handle=h)  # noqa: E731
    fn()
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        fn()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    kernel_ms = ev0.elapsed_time(ev1) / args.steps
    log(f"[bench] batched graph: {sec * 1e3:.3f} ms/step, {flops / sec / 1e12:.2f} TFLOP/s")
    got = out.cpu().numpy()
    # per-matrix launch loop (same kernels, one launch per product)
    loop_out = torch.empty_like(A)
    ns.ns_eval_batched_loop(A, torch.from_numpy(offs), nh, k, "radix9", "f32", out_packed=loop_out, handle=h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loop_steps = 2
    for _ in range(loop_steps):
        ns.ns_eval_batched_loop(A, torch.from_numpy(offs), nh, k, "radix9", "f32", out_packed=loop_out, handle=h)
    torch.cuda.synchronize()
    loop_sec = (time.perf_counter() - t0) / loop_steps
    log(f"[bench] per-matrix loop: {loop_sec * 1e3:.1f} ms/step")
    bit_identical = bool(torch.equal(out, loop_out))

    def oracle_all():
        return [series.radix9(M.astype(np.float32).astype(np.float64), k)[0] for M in w.mats]
    cpu, worst = None, None
    if not args.no_cpu_baseline:
        refs, cpu = cpu_oracle_sample(oracle_all, "whole batch once: radix-9 S_81 of all 2048 matrices",
                                      flops)
        worst = max(series.rel_fro(got[o:o + m * m].reshape(m, m), r)
                    for o, m, r in zip(offs, w.ns, refs))
    line = base_line(args, flops / sec / 1e12, sec * 1e3, "f32",
                     {"workload": "jacobi_batch", "batch": len(w.mats), "n": "U{8..256}", "k": k,
                      "method": "radix9", "products_per_matrix": 10, "seed": w.seed,
                      "total_flops": flops})
    line["loop_ms_per_step"] = round(loop_sec * 1e3, 3)
    line["speedup_over_launch_loop"] = round(loop_sec / sec, 2)
    line["bit_identical_to_launch_loop"] = bit_identical
    line["worst_rel_err_vs_oracle"] = worst
    line["autotune_configs_timed"] = timed
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    line["roofline"] = {"bound": "mfma", "kernel": "batched_kernel (persistent, one launch)",
                        "achieved": round(achieved, 3), "peak": PEAK["f32"], "unit": "TFLOP/s",
                        "frac": round(achieved / PEAK["f32"], 4), "traffic": None,
                        "per_launch_flops": flops, "avg_launch_ms": round(kernel_ms, 5), "launches": args.steps}
    line["cpu_baseline"] = cpu
    return line


def bench_small_symmetric(args, torch, ns):
    """n = 256 FP64, k = 81: naive (80 products), binary (14), radix-9 (10)."""
    import workloads
    from oracle import series
    w = workloads.make("small_symmetric")
    n, k = 256, 81
    h = ns.Handle(0)
    stream = torch.cuda.current_stream()
    A = torch.from_numpy(w.A).cuda()
    out = torch.empty_like(A)
    res, errs = {}, {}
    for method in ("radix9", "binary", "naive"):
        res[method] = time_leg(ns, h, A, k, method, "f64", out, max(args.steps, 20), args.warmup, stream, n,
                               separate_events=True)
        ref = series.spectral_form(w.Q, w.lam, res[method]["k_eff"])
        errs[method] = series.rel_fro(out.cpu().numpy(), ref)
    main = res["radix9"]
    cpu = None
    if not args.no_cpu_baseline:
        reps = 200
        _, cpu = cpu_oracle_sample(lambda: [series.radix9(w.A, k) for _ in range(reps)],
                                   f"radix-9 S_81 at n=256 repeated {reps} times", reps * 10 * 2.0 * n ** 3)
    line = base_line(args, main["tflops"], main["ms"], "f64",
                     {"workload": "small_symmetric", "n": n, "k": k, "method": "radix9", "seed": w.seed})
    line["legs"] = {m: {**rnd(r), "rel_err_vs_closed_form": errs[m]} for m, r in res.items()}
    line["roofline"] = roofline_from_leg(main, n, "gemm_f64_splitk_kernel", "f64")
    line["cpu_baseline"] = cpu
    return line


WORKLOADS = {
    "large_symmetric": bench_large_symmetric,
    "gaussian_rho": bench_gaussian_rho,
    "precision_sym": bench_precision_sym,
    "jacobi_batch": bench_jacobi_batch,
    "small_symmetric": bench_small_symmetric,
}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 2
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import paper_2602_11843_amd as ns
    if args.calibrate_copy_mib:
        nbytes = args.calibrate_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calibrate_copy_mib} MiB done")
    names = list(WORKLOADS) if args.workload == "all" else [args.workload]
    for name in names:
        line = WORKLOADS[name](args, torch, ns)
        print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
