"""GPU parity of the mixed-precision forms against the FP64 oracle.

Mixed forms read A in FP64, run the bulk products as FP32, split-BF16 (three
BF16 products) or scaled FP16 on the matrix cores with FP32 accumulation, and
keep FP64 for the running sum (S or Y) and, in the residual methods, for the
residual product R = I - (I - A) Y.  Bars (relative Frobenius error against
the FP64 oracle of the same method): FP32 1e-5, split-BF16 1e-4; scaled FP16
has no stated bar and is held to 1e-2 here (its measured error is printed).
"""

import sys

import numpy as np
import pytest

import workloads
from conftest import assert_close
from oracle import series

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f32_acc64": 1e-5, "split_bf16": 1e-4, "f16_scaled": 1e-2}


@pytest.fixture(scope="module")
def ns():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_11843_amd as ns
    return ns


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(ns, A, k, method, dtype):
    say(f"[gpu] {method} {dtype} n={A.shape[0]} k={k}")
    out, rep = ns.ns_eval_ex(torch.from_numpy(np.ascontiguousarray(A)).cuda(), k, method, dtype,
                             report=True)
    torch.cuda.synchronize()
    return out.cpu().numpy(), rep


@pytest.mark.parametrize("dtype", ["f32_acc64", "split_bf16", "f16_scaled"])
@pytest.mark.parametrize("method", ["binary", "radix9", "quinary", "radix15", "radix9_resid", "hensel",
                                    "radix15c", "mixed"])
@pytest.mark.parametrize("n", [64, 300])
def test_mixed_precision_parity(ns, method, dtype, n):
    w = workloads.symmetric(n, 0.9, 200 + n)
    k = 729
    got, rep = run(ns, w.A, k, method, dtype)
    ref, orep = series.evaluate(w.A, k, method)
    assert_close(got, ref, TOL[dtype], f"{method} {dtype} n={n}")
    assert rep["gemms_performed"] == orep["products"]
    assert not rep["nonfinite"]


@pytest.mark.parametrize("dtype", ["f32_acc64", "split_bf16", "f16_scaled"])
@pytest.mark.parametrize("method", ["radix9", "radix9_resid", "radix15"])
def test_mixed_precision_large_tiles(ns, method, dtype):
    """n = 2048 runs the large-tile engines (the n = 8192 workload's kernels)."""
    w = workloads.symmetric(2048, 0.9, 4)
    k = 729 if method != "radix15" else 3375
    got, rep = run(ns, w.A, k, method, dtype)
    assert_close(got, series.spectral_form(w.Q, w.lam, rep["k_eff"]), TOL[dtype],
                 f"{method} {dtype} n=2048")


def test_residual_form_corrects_low_precision(ns):
    """The residual iteration with an FP64 residual recovers accuracy the
    telescoping form cannot: its error is far below the FP16 products'."""
    w = workloads.symmetric(300, 0.9, 9)
    tele, _ = run(ns, w.A, 729, "radix9", "f16_scaled")
    resid, _ = run(ns, w.A, 729, "radix9_resid", "f16_scaled")
    ref, _ = series.radix9(w.A, 729)
    e_t, e_r = series.rel_fro(tele, ref), series.rel_fro(resid, ref)
    say(f"   telescoping {e_t:.3e}  residual {e_r:.3e}")
    assert e_r < e_t / 10


@pytest.mark.parametrize("dtype", ["f32_acc64", "split_bf16", "f16_scaled"])
@pytest.mark.parametrize("method", ["radix9", "radix9_resid"])
@pytest.mark.parametrize("n", [300, 2048])
def test_mixed_precision_nonsymmetric(ns, method, dtype, n):
    """A nonsymmetric input: every product X Y of the schedule differs from
    X Y^T, so a row/column mix-up of either operand (n = 2048 runs the
    16-bit panel engines, whose Y operand is laid out by columns) fails."""
    g = workloads.gaussian(n, 0.5, 300 + n)
    got, rep = run(ns, g.A, 81, method, dtype)
    ref, orep = series.evaluate(g.A, 81, method)
    assert_close(got, ref, TOL[dtype], f"{method} {dtype} nonsymmetric n={n}")
    assert rep["gemms_performed"] == orep["products"]


@pytest.mark.parametrize("dtype", ["f32_acc64", "split_bf16", "f16_scaled"])
@pytest.mark.parametrize("n", [300, 2048])
def test_mixed_any_k_precision_forms(ns, dtype, n):
    """Exact any-k plans in the precision forms: the FP64 running sum takes
    the additive steps too (S64 += A^n), including the fused last one."""
    g = workloads.gaussian(n, 0.5, 500 + n)
    for k in (2, 4, 10, 100, 1000):
        got, rep = run(ns, g.A, k, "mixed", dtype)
        ref, orep = series.mixed(g.A, k)
        assert_close(got, ref, TOL[dtype], f"mixed {dtype} k={k}")
        assert rep["gemms_performed"] == orep["products"] and rep["k_eff"] == k


@pytest.mark.parametrize("dtype,n,n_internal", [
    ("split_bf16", 2100, 2176), ("split_bf16", 3100, 3328),
    ("f16_scaled", 1700, 1728), ("f16_scaled", 2100, 2304)])
def test_low_precision_padding(ns, dtype, n, n_internal):
    """Padded matrices on both paths of each 16-bit form: below its panel
    threshold (split-BF16 3072, FP16 1792) the operands are converted in the
    k-loop (64-wide tiles, padded to the larger of 64 and the FP64 tile:
    2176 at 2100, 1728 at 1700); from it the products run from panels
    (256-wide padding: 3328, 2304).  The padding block must stay exactly zero
    through every product."""
    w = workloads.symmetric(n, 0.9, 31)
    got, rep = run(ns, w.A, 81, "radix9", dtype)
    assert rep["n_internal"] == n_internal
    assert_close(got, series.spectral_form(w.Q, w.lam, 81), TOL[dtype], f"radix9 {dtype} n={n}")


@pytest.mark.parametrize("n", [64, 2560])
def test_f16_scaled_tiny_operands_stay_finite(ns, n):
    """Operands whose max-abs lies far below FP16's range (here ~1e-36, an FP32
    normal): the operand scale is capped at 2^114 and the product is unscaled
    with ldexp, so no scale overflows and the result is I + A to FP16
    accuracy.  n = 64 converts in the k-loop, n = 2560 runs from panels.
    Binary at k = 4: S = I + A + A^2 + A^3, whose last two terms underflow."""
    w = workloads.symmetric(n, 0.9, 61)
    A = w.A * 1e-36
    got, rep = run(ns, A, 4, "binary", "f16_scaled")
    assert np.all(np.isfinite(got)) and not rep["nonfinite"]
    # off the diagonal S - I is A itself (on it, 1 + A_ii rounds to 1 in FP64)
    off = ~np.eye(n, dtype=bool)
    fro = series.rel_fro(got[off], A[off])
    say(f"   off-diagonal S vs A rel err {fro:.3e}")
    assert fro < TOL["f16_scaled"]
    assert np.array_equal(np.diag(got), np.ones(n))
