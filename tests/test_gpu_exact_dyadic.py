"""Bit-for-bit parity of every product engine and kernel family on inputs
where floating-point arithmetic is exact.

``workloads.dyadic`` inputs (entries k/8, at most three per row and column)
keep every operand of the k = 4 schedules of binary splitting, Horner and
Hensel (I, A, I + A, A^2, A^4) within 8 significant bits, and every product
and sum on a coarse dyadic grid (the premise is pinned on the host in
``test_dyadic_exact.py``).  So the FP64, FP32, split-BF16 (its low parts are
zero), scaled-FP16 (the scales are powers of two) and int8-slice products are
all exact, and S_4(A) = I + A + A^2 + A^3 must come out of every dtype equal
to the FP64 oracle's in every element -- a wrong fragment, k-slab, tile or
epilogue term anywhere shows up as a nonzero difference, however small.

Sizes pick the kernel families: n = 300 the small tiles (16-bit operands
converted in the k-loop); n = 2600 (padded to 2816) the FP64 128 x 128 tile
and the scaled-FP16 panel product with a ragged tail; n = 3072 the split-BF16
panel product; n = 4096 the FP32 128 x 256 tile.
"""

import sys

import numpy as np
import pytest

import workloads
from oracle import series

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ns():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_11843_amd as ns
    return ns


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_cache = {}


def case(n):
    if n not in _cache:
        A = workloads.dyadic(n, 100 + n)
        ref, _ = series.evaluate(A, 4, "binary")          # exact: S_4 = I + A + A^2 + A^3
        _cache[n] = (A, ref)
    return _cache[n]


DTYPES = ["f64", "f32", "f32_acc64", "split_bf16", "f16_scaled"]
# padded sizes of the panel paths (multiples of 256 from n = 1792 for FP16 and
# n = 3072 for split-BF16)
PANEL = {(2600, "f16_scaled"): 2816, (3072, "f16_scaled"): 3072, (3072, "split_bf16"): 3072}


@pytest.mark.parametrize("n", [300, 2600, 3072, 4096])
@pytest.mark.parametrize("method", ["binary", "naive", "hensel"])
def test_every_engine_exact(ns, n, method):
    A, ref = case(n)
    # naive Horner has no FP64-accumulated form (the library refuses it)
    for dtype in (DTYPES if method != "naive" else ["f64", "f32"]):
        say(f"[gpu] exact dyadic {method} {dtype} n={n}")
        Ad = torch.from_numpy(A.astype(np.float32) if dtype == "f32" else A).cuda()
        out, rep = ns.ns_eval_ex(Ad, 4, method, dtype, report=True)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        bad = int(np.count_nonzero(got != ref))
        assert bad == 0, (method, dtype, n, bad, float(np.max(np.abs(got - ref))))
        assert not rep["nonfinite"] and rep["k_eff"] == 4
        if (n, dtype) in PANEL:            # the 16-bit panel products are the ones taken
            assert rep["n_internal"] == PANEL[(n, dtype)]


@pytest.mark.parametrize("n", [300, 3072])
@pytest.mark.parametrize("dtype", ["f32_acc64+i8", "split_bf16+i8", "f16_scaled+i8+last",
                                   "split_bf16+i8x6", "split_bf16+crt", "f32_acc64+crt+last"])
def test_int8_residual_exact(ns, n, dtype):
    """Hensel's residual product through the int8 slices: the digits of A's
    rows and Y's columns hold their values exactly, so the emulated FP64
    product is exact too."""
    A, ref = case(n)
    say(f"[gpu] exact dyadic hensel {dtype} n={n}")
    out, rep = ns.ns_eval_ex(torch.from_numpy(A).cuda(), 4, "hensel", dtype, report=True)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(got, ref), (dtype, n, int(np.count_nonzero(got != ref)))
    # the last residual is A^4 exactly (Lemma 5.9: R_n = E^[n](A) for Hensel, E(x) = x^2)
    A2 = A @ A
    assert rep["level_norm"][1] == pytest.approx(np.linalg.norm(A2 @ A2), rel=1e-15)
