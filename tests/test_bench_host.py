"""Host-side checks of the benchmark's measurement logic (no GPU): the
per-launch roofline arithmetic, the counter-traffic lookup and its source
hash, the CPU sample loop, the one-GPU guard and the residual measure."""

import hashlib
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402

HASHED = bench.KERNEL_SOURCES


def test_engine_roofline_uses_logged_flops_per_launch():
    n = 4096
    stats = (150, 150 * 2.0, 150 * 2.0 * n ** 3)        # launches, summed ms, summed flops
    r = bench.engine_roofline("f64", stats, n)
    assert r["achieved"] == pytest.approx(2.0 * n ** 3 / 2e-3 / 1e12, rel=1e-4)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6, rel=1e-3)
    assert r["peak"] == 78.6 and r["bound"] == "mfma" and r["launches"] == 150
    assert r["avg_launch_ms"] == pytest.approx(2.0)
    assert r["kernel"] == "gemm_kernel<PolF64M16<2,2,4,4>>"
    # three BF16 MFMA products per logical product (split-BF16), BF16 peak
    r3 = bench.engine_roofline("split_bf16", stats, n)
    assert r3["achieved"] == pytest.approx(3 * r["achieved"], rel=1e-4)
    assert r3["peak"] == 2516.6
    # a launch carrying two products logs twice the flops
    r2 = bench.engine_roofline("f64", (75, 300.0, 150 * 2.0 * n ** 3), n)
    assert r2["achieved"] == pytest.approx(r["achieved"], rel=1e-4)
    assert r2["per_launch_flops"] == pytest.approx(2 * 2.0 * n ** 3)
    assert bench.engine_roofline("f64", (0, 0.0, 0.0), n) is None


def test_kernel_names_follow_the_tile_thresholds():
    assert bench.kernel_name("f64", 256) == "gemm_f64_splitk_kernel"
    assert bench.kernel_name("f64", 1024) == "gemm_kernel<PolF64M16<2,2,1,1,4>>"
    assert bench.kernel_name("f32", 8192) == "gemm_kernel<PolF32<2,2,4,8>>"
    assert bench.kernel_name("f32", 2048) == "gemm_kernel<PolF32<2,2,2,2>>"
    assert "PolPanel" in bench.kernel_name("split_bf16", 8192)
    assert "PolLow" in bench.kernel_name("f16_scaled", 1536)
    assert "PolPanel" in bench.kernel_name("f16_scaled", 2048)


def test_int8_products_per_residual():
    """The roofline of the emulated residual counts s (s + 1) / 2 int8
    products for the digit form and one per modulus for the residue form."""
    assert bench.i8_products("split_bf16+i8", 8192) == 28
    assert bench.i8_products("split_bf16+i8x6+last", 8192) == 21
    assert bench.i8_products("split_bf16+crt+last", 8192) == 14
    assert bench.i8_products("split_bf16+crt", 256) == 13
    assert bench.i8_products("split_bf16+last", 8192) == 0


def _fake_root(tmp_path, traffic=123456789):
    csrc = tmp_path / "paper_2602_11843_amd" / "csrc"
    csrc.mkdir(parents=True)
    h = hashlib.sha256()
    for f in HASHED:
        src = os.path.join(ROOT, "paper_2602_11843_amd", "csrc", f)
        shutil.copy(src, csrc / f)
        with open(src, "rb") as fh:
            h.update(fh.read())
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "s.md").write_text(
        f"text\n```\nsource_sha256_16 {h.hexdigest()[:16]}\ntraffic_bytes_per_launch {traffic}\n```\n")
    return csrc


def test_measured_traffic_follows_the_source_hash(tmp_path):
    csrc = _fake_root(tmp_path)
    assert bench.measured_traffic("s.md", root=str(tmp_path)) == 123456789.0
    # any change to the kernel sources voids the counter figure
    with open(csrc / "gemm.hip", "a") as fh:
        fh.write("\n")
    assert bench.measured_traffic("s.md", root=str(tmp_path)) is None
    assert bench.measured_traffic("missing.md", root=str(tmp_path)) is None


def test_cpu_sample_repeats_until_the_bound():
    calls = []
    res, rec = bench.cpu_oracle_sample(lambda: calls.append(1) or len(calls), "probe", 1e12,
                                       min_seconds=0.05, max_runs=7)
    assert res == 1                      # the first run's result is returned
    assert 1 <= len(calls) <= 7
    assert rec["kind"] == "oracle" and rec["unit"] == "TFLOP/s" and rec["cores"] >= 1
    assert f"{len(calls)} run(s)" in rec["sample"]


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)


def test_rounding_keeps_small_errors_visible():
    import bench
    r = bench.rnd({"err": 4.643212e-15, "ms": 244.13781234, "nested": {"e": 7.5881e-11}})
    assert r["err"] == 4.643212e-15 and r["nested"]["e"] == 7.5881e-11
    assert r["ms"] == 244.1378


def test_residual_measure_matches_closed_form():
    """||I - (I - A) S||_F for S = S_k(A) is ||A^k||_F: on a diagonal A with
    entries lam, sqrt(sum lam^(2k)).  Host tensors, FP64."""
    torch = pytest.importorskip("torch")
    lam = np.array([0.5, -0.25, 0.75, 0.0, 0.125])
    k = 9
    A = torch.from_numpy(np.diag(lam))
    S = torch.from_numpy(np.diag((1 - lam ** k) / (1 - lam)))
    want = float(np.sqrt(np.sum(lam ** (2 * k))))
    assert bench.residual_fro(torch, A, S) == pytest.approx(want, rel=1e-12)
    # FP32 inputs are widened, and a non-finite result is reported as None
    assert bench.residual_fro(torch, A.float(), S.float()) == pytest.approx(want, rel=1e-6)
    S[0, 0] = float("inf")
    assert bench.residual_fro(torch, A, S) is None
