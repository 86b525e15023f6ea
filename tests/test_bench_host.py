"""Host-side checks of the benchmark's measurement logic (no GPU): the
per-launch roofline arithmetic, the counter-traffic lookup and its source
hash, the CPU sample loop, and the one-GPU guard."""

import hashlib
import os
import shutil
import subprocess
import sys

import pytest

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402

HASHED = ("gemm_device.h", "gemm.hip", "ns.cpp")


def test_roofline_from_leg_uses_logged_flops_per_launch():
    n = 4096
    leg = {"product_launches": 150, "product_avg_ms": 2.0, "launch_flops": 2.0 * n ** 3}
    r = bench.roofline_from_leg(leg, n, "k", "f64")
    assert r["achieved"] == pytest.approx(2.0 * n ** 3 / 2e-3 / 1e12, rel=1e-4)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6, rel=1e-3)
    assert r["peak"] == 78.6 and r["bound"] == "mfma" and r["launches"] == 150
    # three BF16 MFMA products per logical product (split-BF16)
    r3 = bench.roofline_from_leg(leg, n, "k", "bf16", mfma_per_logical=3.0)
    assert r3["achieved"] == pytest.approx(3 * r["achieved"], rel=1e-4)
    assert bench.roofline_from_leg({"product_launches": 0}, n, "k", "f64") is None


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
    # any change to the kernel or schedule sources voids the counter figure
    with open(csrc / "ns.cpp", "a") as fh:
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
