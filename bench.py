#!/usr/bin/env python3
"""Benchmark: S_k(A) time and GEMM TFLOP/s on one MI355X.

One step = one evaluation of S_k(A).  The headline (the JSON line's `value`)
is the largest single-GPU configuration:

    precision_sym: n = 8192, k = 729 = 9^3, A = Q diag(lam) Q^T with
    lam ~ U[-0.9, 0.9], seed 4; radix-9 (15 products) with every product on
    FP64 MFMA.  Its squaring baseline is binary splitting (20 products,
    k_eff = 1024) in FP64 on the same input.

`value` is logical GEMM TFLOP/s of the headline step: (products x 2 n^3) /
step time, inputs resident in HBM before the timed region.  The line also
carries, measured with the same protocol (warm-up calls, then `steps` timed
calls bracketed by device synchronisation) and each with its own roofline,
the legs of the other workloads:

  precision_sym   radix-9 in FP32, FP32 + FP64 sum, split-BF16, scaled FP16;
                  the residual forms (FP64 residual) in split-BF16, scaled
                  FP16 and FP32; split-BF16 with the residual exact only at
                  the last two levels, or emulated from int8 slices or
                  through residues modulo 14 pairwise-coprime moduli
  gaussian_rho    n = 8192 FP32, nonsymmetric, rho_hat = 0.99, k = 3375:
                  radix-15 (contraction-aware table and App. B table),
                  radix-9 (k_eff 6561), binary (k_eff 4096), the exact any-k
                  plan, and the contraction-aware radix-15 with FP32 products
                  and an FP64 residual; level norms per leg; the App. B
                  table again at rho_hat = 0.95
  large_symmetric n = 4096, k = 729: radix-9 and binary in FP64 and FP32
  jacobi_batch    2048 small FP32 matrices, k = 81 radix-9: one persistent
                  graph launch against the per-matrix launch loop
  small_symmetric n = 256 FP64, k = 81: radix-9, binary, naive; time per
                  product launch and the critical path in launches

Every leg's roofline comes from HIP events recorded by the library around each
product launch on the call's stream, per product engine.  The CPU oracle
(test infrastructure) is timed on a bounded sample on the host's cores.
`--workload NAME` runs one workload and prints its own line.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

METRIC = "S_k(A) time + GEMM TFLOP/s (%MFMA peak), radix-9/15 vs squaring at stated err"
# dense MI355X peaks (TFLOP/s; int8: TOP/s)
PEAK = {"f64": 78.6, "f32": 157.3, "split_bf16": 2516.6, "f16_scaled": 2516.6, "i8": 5000.0}
# MFMA work per logical product on each engine (split-BF16: three BF16 products;
# the int8-emulated residual: its int8 products, set per leg by i8_products)
MFMA_PER_LOGICAL = {"f64": 1.0, "f32": 1.0, "split_bf16": 3.0, "f16_scaled": 1.0}
ENGINES = ("f64", "f32", "split_bf16", "f16_scaled", "i8")


def crt_moduli(n):
    """Moduli of the residue form at padded n (ns.h: their product exceeds
    n 2^94): 13 at n = 256, 14 from 512 to 65536."""
    M, count = 1, 0
    for m in (256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197, 193):
        M *= m
        count += 1
        if M > n << 94:
            return count
    raise ValueError(f"n = {n} beyond the residue form's moduli")


def i8_products(dtype, n):
    """int8 products per emulated residual product of a dtype name: s (s + 1) / 2
    for int8 slices (s = 7 for "+i8"), one per modulus for "+crt"; 0 without."""
    for m in dtype.split("+")[1:]:
        if m == "i8":
            return 28
        if m.startswith("i8x"):
            s = int(m[3:])
            return s * (s + 1) // 2
        if m == "crt":
            return crt_moduli(n)
    return 0


ROOT = os.path.dirname(os.path.abspath(__file__))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="all",
                    choices=["all", "precision_sym", "gaussian_rho", "large_symmetric",
                             "jacobi_batch", "small_symmetric"])
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip timing the CPU oracle (profiling runs)")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the accuracy checks against host references (profiling runs)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    ap.add_argument("--only", default="",
                    help="comma list of method:dtype legs to run (profiling runs)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# rooflines
# ---------------------------------------------------------------------------

def kernel_name(engine, n):
    """The product kernel an engine runs at padded size n."""
    if engine == "f64":
        if n >= 2048:
            return "gemm_kernel<PolF64M16<2,2,4,4>>"
        if 160 <= n <= 256:
            return "gemm_f64_splitk_kernel"
        return "gemm_kernel<PolF64M16<2,2,1,1,4>>"
    if engine == "f32":
        return "gemm_kernel<PolF32<2,2,4,8>>" if n >= 4096 else "gemm_kernel<PolF32<2,2,2,2>>"
    if engine == "split_bf16":
        return ("gemm_panel_kernel<PolPanel<2,4,4,2,true,1,2,2>>" if n >= 3072
                else "gemm_lowp_kernel<PolLow<2,2,1,1,true>>")
    if engine == "i8":
        return "gemm_i8_kernel<PolI8> (one launch per slice diagonal, or per modulus)"
    return ("gemm_panel_kernel<PolPanel<1,4,4,2,false,...,Y in registers>>" if n >= 1792
            else "gemm_lowp_kernel<PolLow<2,2,1,1,false>>")


def engine_roofline(engine, stats, n, i8_per_product=0):
    """Roofline of one engine's product launches: MFMA work per launch (2 n^3
    per logical product, times 3 for split-BF16, times the int8 products of
    one emulated residual product) over the launches' average duration,
    against that engine's dense MFMA peak."""
    cnt, ms, flops = stats
    if not cnt or ms <= 0:
        return None
    mfma = i8_per_product if engine == "i8" else MFMA_PER_LOGICAL[engine]
    achieved = mfma * flops / (ms * 1e-3) / 1e12
    peak = PEAK[engine]
    return {"bound": "mfma", "kernel": kernel_name(engine, n), "achieved": round(achieved, 3),
            "peak": peak, "unit": "TOP/s" if engine == "i8" else "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": None,
            "per_launch_flops": mfma * flops / cnt, "avg_launch_ms": round(ms / cnt, 5),
            "launches": cnt}


KERNEL_SOURCES = ("gemm_device.h", "gemm.hip", "common.h")


def kernel_source_hash(root=None):
    """Hash of the FP64/FP32 product kernels' sources: a counter summary taken
    on other sources no longer describes the kernel."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(root or ROOT, "paper_2602_11843_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(summary, root=None):
    """HBM bytes per launch from a committed rocprofv3 counter summary under
    profiles/, or None when the summary is missing or was taken on other
    kernel sources (it records their hash)."""
    path = os.path.join(root or ROOT, "profiles", summary)
    try:
        vals = {}
        with open(path) as fh:
            for line in fh:
                parts = line.split()
                if len(parts) == 2 and parts[0] in ("source_sha256_16", "traffic_bytes_per_launch"):
                    vals[parts[0]] = parts[1]
        if vals.get("source_sha256_16") != kernel_source_hash(root):
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


# ---------------------------------------------------------------------------
# timing
# ---------------------------------------------------------------------------

def time_leg(ns, h, A, k, method, dtype, out, steps, warmup, stream, n, separate_events=False):
    """Time `steps` evaluations after `warmup`.  Per-launch HIP events on the
    call's stream are recorded during the timed steps; with separate_events
    the timed steps run without them (at small n the event records between
    launches are a visible part of a call) and a second pass of as many steps
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
    per_engine = {e: h.ns_product_timing_dtype(ns.RESID_INT8(0) if e == "i8" else e) for e in ENGINES}
    launches = h.ns_product_timing_launches()
    cnt, kms, kfl = h.ns_product_timing(reset=True)
    h.ns_set_product_timing(False)
    _, rep = ns.ns_eval_ex(A, k, method, dtype, out=out, handle=h, stream=stream, report=True)
    flops = products * 2.0 * n ** 3
    rooflines = {e: engine_roofline(e, st, rep["n_internal"], i8_products(dtype, rep["n_internal"]))
                 for e, st in per_engine.items() if st[0]}
    dominant = max(rooflines, key=lambda e: per_engine[e][1]) if rooflines else None
    # per-level split of the last timed call (its launches are the last ones recorded)
    per_call = rep["product_launches"]
    last = [ms for ms, _ in launches[-per_call:]] if per_call and len(launches) >= per_call else []
    level_ms = None
    if last and levels and per_call % levels == 0:
        per_lv = per_call // levels
        level_ms = [round(sum(last[i * per_lv:(i + 1) * per_lv]), 4) for i in range(levels)]
    r = {"ms": sec * 1e3, "tflops": flops / sec / 1e12, "products": products, "k_eff": k_eff,
         "level_ms_last_call": level_ms,
         "levels": levels, "product_launches_per_call": rep["product_launches"],
         "launches_timed": cnt, "kernel_ms_per_call": kms / steps,
         "roofline": rooflines.get(dominant), "rooflines_by_engine": rooflines,
         "level_norm": rep["level_norm"], "nonfinite": rep["nonfinite"]}
    log(f"[bench]   {sec * 1e3:.3f} ms/step  {flops / sec / 1e12:.2f} TFLOP/s logical; "
        + "; ".join(f"{e} {v['avg_launch_ms']:.4f} ms/launch {v['frac']:.3f} of peak"
                    for e, v in rooflines.items()))
    return r


def rnd(d):
    """Floats to 7 significant digits (errors of 1e-15 stay visible)."""
    out = {}
    for k, v in d.items():
        if isinstance(v, float):
            out[k] = float(f"{v:.7g}")
        elif isinstance(v, dict):
            out[k] = rnd(v)
        else:
            out[k] = v
    return out


def select(legs, args):
    if not args.only:
        return legs
    want = [tuple(x.split(":")) for x in args.only.split(",")]
    return [l for l in legs if l[:2] in want]


# ---------------------------------------------------------------------------
# CPU oracle baseline
# ---------------------------------------------------------------------------

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


def close(got, ref):
    """(relative Frobenius error, max element error / max |ref|)."""
    d = np.asarray(got, np.float64) - ref
    return (float(np.linalg.norm(d) / np.linalg.norm(ref)),
            float(np.max(np.abs(d)) / np.max(np.abs(ref))))


def residual_fro(torch, A, S):
    """||I - (I - A) S||_F, the accuracy measure of Sec. 6, in FP64 from the
    call's input A and output S (device or host tensors).  A check of the
    result, computed with torch.matmul outside the timed region."""
    A64, S64 = A.double(), S.double()
    R = S64 - torch.matmul(A64, S64)
    R.diagonal().sub_(1.0)
    v = float(torch.linalg.norm(R))
    del R, A64, S64
    return v if math.isfinite(v) else None


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def bench_precision_sym(args, torch, ns):
    """n = 8192, k = 729, symmetric lam ~ U[-0.9, 0.9]: radix-9 with every
    product in FP64 (the headline) against binary splitting in FP64, and
    radix-9 in the precision forms."""
    import workloads
    from oracle import series                      # benchmark infrastructure only
    log("[bench] generating precision_sym input (n=8192)")
    w = workloads.make("precision_sym")
    n, k = w.A.shape[0], 729
    ref = None if args.no_check else series.spectral_form(w.Q, w.lam, k)
    ref_bin = None if args.no_check else series.spectral_form(w.Q, w.lam, 1024)
    h = ns.Handle(0)
    stream = torch.cuda.current_stream()
    A64 = torch.from_numpy(w.A).cuda()
    A32 = A64.float()
    out64, out32 = torch.empty_like(A64), torch.empty_like(A32)
    legs = select([("radix9", "f64"), ("binary", "f64"), ("radix9", "f32"), ("radix9", "f32_acc64"),
                   ("radix9", "split_bf16"), ("radix9", "f16_scaled"),
                   ("radix9_resid", "split_bf16"), ("radix9_resid", "f16_scaled"),
                   ("radix9_resid", "f32_acc64"),
                   # the residual product exact only at the last two levels, or
                   # emulated from int8 slices (s = 7, 6) or through residues
                   ("radix9_resid", "split_bf16+last"), ("radix9_resid", "split_bf16+i8"),
                   ("radix9_resid", "split_bf16+i8x6"), ("radix9_resid", "split_bf16+i8+last"),
                   ("radix9_resid", "split_bf16+crt"), ("radix9_resid", "split_bf16+crt+last")],
                  args)
    res = {}
    for method, dtype in legs:
        A, out = (A32, out32) if dtype == "f32" else (A64, out64)
        r = time_leg(ns, h, A, k, method, dtype, out, args.steps, args.warmup, stream, n)
        if ref is not None:
            got = out.double().cpu().numpy()
            r["rel_err_vs_definition"], r["max_elem_err_vs_definition"] = close(
                got, ref_bin if method == "binary" else ref)
            del got
            r["residual_fro"] = residual_fro(torch, A, out)
            log(f"[bench]   rel err vs FP64 definition {r['rel_err_vs_definition']:.3e}, "
                f"||I - (I - A) S||_F {r['residual_fro']:.3e}")
        res[f"{method}:{dtype}"] = r
    cpu = None
    if not args.no_cpu_baseline:
        _, cpu = cpu_oracle_sample(lambda: series.radix9(w.A, 9),
                                   "one radix-9 level of the oracle at n=8192 (5 float64 products)",
                                   5 * 2.0 * n ** 3)
    del A64, A32, out64, out32
    h.close()
    torch.cuda.empty_cache()
    info = {"workload": "precision_sym", "n": n, "k": k, "seed": w.seed, "lam": "U[-0.9,0.9]"}
    return res, cpu, info


def bench_gaussian_rho(args, torch, ns):
    """n = 8192 FP32, nonsymmetric N(0,1)/sqrt(n) scaled to rho_hat = 0.99,
    k = 3375: radix-15 (contraction-aware and App. B tables, 18 products)
    against radix-9 (20, k_eff 6561), binary (24, k_eff 4096) and the exact
    any-k plan (19); the contraction-aware radix-15 with FP32 products and an
    FP64 residual; the App. B table again at rho_hat = 0.95."""
    import scipy.linalg
    import workloads
    log("[bench] generating gaussian_rho input (n=8192, 400 power iterations)")
    g = workloads.make("gaussian_rho")
    n, k = g.A.shape[0], 3375
    h = ns.Handle(0)
    stream = torch.cuda.current_stream()
    cols = np.sort(np.random.default_rng(0).choice(n, 16, replace=False))
    I_cols = np.zeros((n, len(cols)))
    I_cols[cols, np.arange(len(cols))] = 1.0
    out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    out64 = None
    res = {}
    for rho in (0.99, 0.95):
        A = g.A * (rho / 0.99)
        refs = {}
        if not args.no_check:
            # S_inf columns (I - A)^{-1} e_j, for the FP32-rounded A (what the
            # FP32 path receives) and the FP64 A; A^k is below 1e-8 here
            for prec in ("f32", "f64"):
                Ap = A.astype(np.float32).astype(np.float64) if prec == "f32" else A
                log(f"[bench] LU reference (I - A)^-1 e_j for rho {rho} ({prec} input)")
                refs[prec] = scipy.linalg.lu_solve(scipy.linalg.lu_factor(np.eye(n) - Ap), I_cols)
        A32 = torch.from_numpy(A).float().cuda()
        A64 = torch.from_numpy(A).cuda()
        legs = ([("radix15c", "f32"), ("radix15", "f32"), ("radix9", "f32"), ("binary", "f32"),
                 ("mixed", "f32"), ("radix15c", "f32_acc64")] if rho == 0.99 else [("radix15", "f32")])
        for method, dtype in select(legs, args):
            if dtype == "f32":
                Ad, o = A32, out
            else:
                out64 = out64 if out64 is not None else torch.empty((n, n), dtype=torch.float64,
                                                                    device="cuda")
                Ad, o = A64, out64
            r = time_leg(ns, h, Ad, k, method, dtype, o, args.steps, args.warmup, stream, n)
            if refs:
                got = o[:, torch.from_numpy(cols).cuda()].double().cpu().numpy()
                r["rel_err_sampled_vs_inverse"], r["max_elem_err_sampled_vs_inverse"] = close(
                    got, refs["f32" if dtype == "f32" else "f64"])
                r["residual_fro"] = residual_fro(torch, Ad, o)
                log(f"[bench]   rho {rho} {method} {dtype}: sampled rel err vs (I-A)^-1 "
                    f"{r['rel_err_sampled_vs_inverse']:.3e}, level norms "
                    f"{['%.3g' % x for x in r['level_norm']]}")
            res[f"{method}:{dtype}:rho{rho}"] = r
        del A32, A64
    h.close()
    del out, out64
    torch.cuda.empty_cache()
    info = {"workload": "gaussian_rho", "n": n, "k": k, "rho_hat": 0.99, "seed": g.seed}
    return res, None, info


def bench_large_symmetric(args, torch, ns):
    """n = 4096, k = 729: radix-9 against binary in FP64 and FP32."""
    import workloads
    from oracle import series
    w = workloads.make("large_symmetric")
    n, k = w.A.shape[0], 729
    h = ns.Handle(0)
    stream = torch.cuda.current_stream()
    A64 = torch.from_numpy(w.A).cuda()
    A32 = A64.float()
    out64, out32 = torch.empty_like(A64), torch.empty_like(A32)
    legs = select([("radix9", "f64"), ("binary", "f64"), ("radix9", "f32"), ("binary", "f32")], args)
    cols = np.sort(np.random.default_rng(0).choice(n, 64, replace=False))
    res = {}
    for method, dtype in legs:
        A, out = (A64, out64) if dtype == "f64" else (A32, out32)
        r = time_leg(ns, h, A, k, method, dtype, out, args.steps, args.warmup, stream, n)
        if not args.no_check:
            got = out[:, torch.from_numpy(cols).cuda()].double().cpu().numpy()
            ref = series.spectral_form(w.Q, w.lam, r["k_eff"], cols=cols)
            r["rel_err_sampled_vs_definition"], _ = close(got, ref)
            r["residual_fro"] = residual_fro(torch, A, out)
        res[f"{method}:{dtype}"] = r
    h.close()
    info = {"workload": "large_symmetric", "n": n, "k": k, "seed": w.seed, "lam": "U[-0.95,0.95]"}
    return res, None, info


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
    out = torch.empty_like(A)
    k = 81
    flops = float(sum(10 * 2.0 * int(m) ** 3 for m in w.ns))
    h = ns.Handle(0)
    # the autotuner's pick is also written to this JSON-lines file
    os.environ.setdefault("NS_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "ns_tune.jsonl"))
    log("[bench] autotuning the batched kernel")
    timed = ns.ns_autotune_batched(A, offd, None, nh, k, out, handle=h)
    log(f"[bench]   {timed} configurations timed")
    fn = lambda: ns.ns_eval_batched(A, offd, None, nh, k, "radix9", "f32", out_packed=out, handle=h)  # noqa: E731
    fn()
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        fn()
    torch.cuda.synchronize()
    # the graph runs on the current stream, so torch's events see its kernel
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
    loop_out = torch.empty_like(A)
    offs_t = torch.from_numpy(offs)
    ns.ns_eval_batched_loop(A, offs_t, nh, k, "radix9", "f32", out_packed=loop_out, handle=h)
    torch.cuda.synchronize()
    loop_steps = max(5, args.steps // 4)
    t0 = time.perf_counter()
    for _ in range(loop_steps):
        ns.ns_eval_batched_loop(A, offs_t, nh, k, "radix9", "f32", out_packed=loop_out, handle=h)
    torch.cuda.synchronize()
    loop_sec = (time.perf_counter() - t0) / loop_steps
    log(f"[bench] per-matrix loop: {loop_sec * 1e3:.1f} ms/step over {loop_steps} steps")
    bit_identical = bool(torch.equal(out, loop_out))
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    r = {"ms": sec * 1e3, "tflops": flops / sec / 1e12, "products_per_matrix": 10,
         "batch": len(w.mats), "total_flops": flops, "loop_ms": loop_sec * 1e3,
         "loop_steps": loop_steps, "speedup_over_launch_loop": loop_sec / sec,
         "bit_identical_to_launch_loop": bit_identical, "autotune_configs_timed": timed,
         "roofline": {"bound": "mfma", "kernel": "batched_kernel (persistent, one launch)",
                      "achieved": round(achieved, 3), "peak": PEAK["f32"], "unit": "TFLOP/s",
                      "frac": round(achieved / PEAK["f32"], 4), "traffic": None,
                      "per_launch_flops": flops, "avg_launch_ms": round(kernel_ms, 5),
                      "launches": args.steps}}
    cpu = None
    if not args.no_check:
        def oracle_all():
            return [series.radix9(M.astype(np.float32).astype(np.float64), k)[0] for M in w.mats]
        if args.no_cpu_baseline:
            refs = oracle_all()
        else:
            refs, cpu = cpu_oracle_sample(oracle_all, "whole batch once: radix-9 S_81 of all 2048 matrices",
                                          flops, min_seconds=3.0)
        r["worst_rel_err_vs_oracle"] = max(series.rel_fro(got[o:o + m * m].reshape(m, m), ref)
                                           for o, m, ref in zip(offs, w.ns, refs))
        r["cpu_baseline"] = cpu
    h.close()
    info = {"workload": "jacobi_batch", "batch": len(w.mats), "n": "U{8..256}", "k": k,
            "seed": w.seed}
    return {"radix9:f32:batched": r}, cpu, info


def bench_small_symmetric(args, torch, ns):
    """n = 256 FP64, k = 81: naive (80 products), binary (14), radix-9 (10).
    Latency-bound: per-launch time and the critical path in launches."""
    import workloads
    from oracle import series
    w = workloads.make("small_symmetric")
    n, k = 256, 81
    h = ns.Handle(0)
    stream = torch.cuda.current_stream()
    A = torch.from_numpy(w.A).cuda()
    out = torch.empty_like(A)
    res = {}
    for method, dtype in select([("radix9", "f64"), ("binary", "f64"), ("naive", "f64")], args):
        r = time_leg(ns, h, A, k, method, dtype, out, max(args.steps, 20), args.warmup, stream, n,
                     separate_events=True)
        r["us_per_product"] = r["ms"] * 1e3 / r["products"]
        r["us_per_launch_on_critical_path"] = r["ms"] * 1e3 / r["product_launches_per_call"]
        if not args.no_check:
            r["rel_err_vs_closed_form"], _ = close(out.cpu().numpy(),
                                                   series.spectral_form(w.Q, w.lam, r["k_eff"]))
            r["residual_fro"] = residual_fro(torch, A, out)
        res[f"{method}:{dtype}"] = r
    cpu = None
    if not args.no_cpu_baseline:
        reps = 100
        _, cpu = cpu_oracle_sample(lambda: [series.radix9(w.A, k) for _ in range(reps)],
                                   f"radix-9 S_81 at n=256 repeated {reps} times", reps * 10 * 2.0 * n ** 3,
                                   min_seconds=3.0)
        res["radix9:f64"]["cpu_baseline"] = cpu
    h.close()
    info = {"workload": "small_symmetric", "n": n, "k": k, "seed": w.seed, "lam": "U[-0.5,0.5]"}
    return res, cpu, info


WORKLOADS = {
    "precision_sym": bench_precision_sym,
    "gaussian_rho": bench_gaussian_rho,
    "large_symmetric": bench_large_symmetric,
    "jacobi_batch": bench_jacobi_batch,
    "small_symmetric": bench_small_symmetric,
}

# the headline leg of each workload when it runs alone
MAIN_LEG = {"precision_sym": "radix9:f64", "gaussian_rho": "radix15c:f32:rho0.99",
            "large_symmetric": "radix9:f64", "jacobi_batch": "radix9:f32:batched",
            "small_symmetric": "radix9:f64"}


def vendor_reference(torch, n=8192, reps=10):
    """The vendor BLAS on the same part, as a practical ceiling beside each
    engine's roofline: torch.matmul of two n x n matrices per precision (and
    torch._int_mm for int8), event-timed on the current stream.  Run only;
    nothing of it is used by the library."""
    out = {}
    cases = [("f64", torch.float64, PEAK["f64"]), ("f32", torch.float32, PEAK["f32"]),
             ("bf16", torch.bfloat16, PEAK["split_bf16"]), ("f16", torch.float16, PEAK["f16_scaled"]),
             ("i8", torch.int8, PEAK["i8"])]
    for name, dt, peak in cases:
        try:
            if dt == torch.int8:
                a = torch.randint(-127, 128, (n, n), dtype=dt, device="cuda")
                b = torch.randint(-127, 128, (n, n), dtype=dt, device="cuda")
                fn = lambda: torch._int_mm(a, b)          # noqa: E731
            else:
                a = torch.randn((n, n), device="cuda").to(dt)
                b = torch.randn((n, n), device="cuda").to(dt)
                fn = lambda: torch.matmul(a, b)           # noqa: E731
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            rate = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
            out[name] = {"ms": round(ms, 4), "rate": round(rate, 2), "unit": "TOP/s" if name == "i8" else "TFLOP/s",
                         "frac_of_peak": round(rate / peak, 4)}
            log(f"[bench] vendor {name} n={n}: {ms:.3f} ms, {rate:.1f} ({rate / peak:.3f} of peak)")
            del a, b
        except Exception as e:                            # noqa: BLE001  (a missing vendor path)
            out[name] = {"error": str(e)[:120]}
    torch.cuda.empty_cache()
    return out


def speedups(res, pairs):
    """wall-time ratio of the squaring leg over each radix leg, beside the
    product-count prediction."""
    out = {}
    for fast, slow in pairs:
        if fast in res and slow in res:
            out[f"{fast} over {slow}"] = {
                "measured": round(res[slow]["ms"] / res[fast]["ms"], 4),
                "predicted_by_product_count": round(res[slow]["products"] / res[fast]["products"], 4)}
    return out


def build_line(args, name, res, cpu, info):
    main_key = MAIN_LEG[name] if MAIN_LEG[name] in res else next(iter(res))
    main = res[main_key]
    dtype = main_key.split(":")[1]
    line = {"metric": METRIC, "value": round(main["tflops"], 4), "unit": "TFLOP/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(main["ms"], 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic",
            "config": {**info, "method": main_key.split(":")[0],
                       "k_eff": main.get("k_eff"), "products": main.get("products")}}
    line["pct_mfma_peak"] = round(100.0 * main["tflops"] / PEAK.get(dtype, PEAK["f32"]), 2)
    line["roofline"] = main.get("roofline")
    return line, main_key


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 2
    sys.path.insert(0, ROOT)
    import paper_2602_11843_amd as ns
    if args.calibrate_copy_mib:
        nbytes = args.calibrate_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"[bench] calibration copy of {args.calibrate_copy_mib} MiB done")

    if args.workload != "all":
        res, cpu, info = WORKLOADS[args.workload](args, torch, ns)
        line, main_key = build_line(args, args.workload, res, cpu, info)
        line["legs"] = {k: rnd(v) for k, v in res.items()}
        line["cpu_baseline"] = cpu
        print(json.dumps(line), flush=True)
        return 0

    # the headline workload first, then every other workload as legs
    res, cpu, info = bench_precision_sym(args, torch, ns)
    line, main_key = build_line(args, "precision_sym", res, cpu, info)
    if line["roofline"] is not None and main_key == "radix9:f64":
        line["roofline"]["traffic"] = measured_traffic("pmc_gemm_f64_big_precision_sym.md")
        line["roofline"]["traffic_unit"] = ("bytes per launch between L2 and the memory side (MALL or HBM): "
                                           "FETCH_SIZE + WRITE_SIZE, copy-calibrated")
    line["cpu_baseline"] = cpu
    legs = {f"precision_sym/{k}": rnd(v) for k, v in res.items()}
    line["speedup_over_binary"] = speedups(res, [("radix9:f64", "binary:f64")])
    for name in ("gaussian_rho", "large_symmetric", "jacobi_batch", "small_symmetric"):
        r, _, _ = WORKLOADS[name](args, torch, ns)
        legs.update({f"{name}/{k}": rnd(v) for k, v in r.items()})
        if name == "gaussian_rho":
            line["speedup_over_binary_gaussian_rho"] = speedups(
                r, [(f"{m}:f32:rho0.99", "binary:f32:rho0.99") for m in ("radix15c", "radix15", "radix9",
                                                                         "mixed")])
        if name == "large_symmetric":
            line["speedup_over_binary_large_symmetric"] = speedups(
                r, [("radix9:f64", "binary:f64"), ("radix9:f32", "binary:f32")])
        if name == "small_symmetric":
            line["speedup_over_binary_small_symmetric"] = speedups(r, [("radix9:f64", "binary:f64")])
    line["legs"] = legs
    line["vendor_gemm_reference_n8192"] = vendor_reference(torch)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
