"""GPU parity of the residual-product variants (NS_RESID_LAST, NS_RESID_INT8,
NS_RESID_CRT) of the FP64-accumulating residual forms (Sec. 5.3, eq. (8)).

Reference: the oracle's FP64 schedule of the same method on the same input.
Bars: every variant within its base dtype's bar (split-BF16 1e-4, FP32 1e-5,
scaled FP16 1e-2), and the accuracy class the variant exists for:

  - int8 slices with s = 7 carry about 2^-49 n relative error in A Y, like
    an FP64 product: the result is within 2x of the FP64-residual form's;
  - s = 6 stays within 1e-9 on these inputs, s = 4 within 1e-5;
  - the residue form has the s = 7 bound (46-bit integers rebuilt exactly):
    within 2x of the FP64-residual form's too;
  - NS_RESID_LAST: the residual the final update uses is exact, so for the
    FP32 and split-BF16 forms the result is within 2x of the FP64-residual
    form's (the scaled-FP16 form loses more: its first residual's error
    inflates the last level's update).
"""

import sys

import numpy as np
import pytest

import workloads
from conftest import assert_close
from oracle import series

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BAR = {"f32_acc64": 1e-5, "split_bf16": 1e-4, "f16_scaled": 1e-2}


@pytest.fixture(scope="module")
def ns():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_11843_amd as ns
    return ns


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def handle(ns):
    h = ns.Handle(torch.cuda.current_device())
    yield h
    h.close()


def run(ns, h, A, k, method, dtype, timing=False):
    say(f"[gpu] {method} {dtype} n={A.shape[0]} k={k}")
    Ad = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    if timing:
        h.ns_set_product_timing(True)
        h.ns_product_timing(reset=True)
    out, rep = ns.ns_eval_ex(Ad, k, method, dtype, handle=h, report=True)
    torch.cuda.synchronize()
    eng = None
    if timing:
        eng = {e: h.ns_product_timing_dtype(e)[0]
               for e in ("f64", "f32", "split_bf16", "f16_scaled", ns.RESID_INT8(0))}
        h.ns_set_product_timing(False)
        h.ns_product_timing(reset=True)
    return out.cpu().numpy(), rep, eng


@pytest.fixture(scope="module")
def case_1000():
    """n = 1000 (padded to 1024: 16 int8 tiles, a ragged tail), k = 729, three
    residual levels."""
    w = workloads.symmetric(1000, 0.9, 7)
    return w, series.radix9_resid(w.A, 729)[0]


@pytest.mark.parametrize("base", ["split_bf16", "f32_acc64", "f16_scaled"])
def test_residual_variants_radix9(ns, handle, case_1000, base):
    w, ref = case_1000
    err = {}
    for mod in ("", "+last", "+i8", "+i8x6", "+i8x4", "+i8+last", "+crt", "+crt+last"):
        got, rep, eng = run(ns, handle, w.A, 729, "radix9_resid", base + mod, timing=True)
        assert rep["gemms_performed"] == 15 and not rep["nonfinite"]
        err[mod] = assert_close(got, ref, BAR[base], f"{base}{mod}")[0]
        # which engine computed the three residual products
        wp = {"split_bf16": "split_bf16", "f32_acc64": "f32", "f16_scaled": "f16_scaled"}[base]
        exact = eng[ns.RESID_INT8(0)] if ("i8" in mod or "crt" in mod) else eng["f64"]
        assert exact == (2 if "last" in mod else 3), (mod, eng)
        assert eng[wp] == 12 + (1 if "last" in mod else 0), (mod, eng)
    assert err["+i8"] <= 2 * err[""] + 1e-13
    assert err["+i8+last"] <= 2 * err["+last"] + 1e-13
    assert err["+crt"] <= 2 * err[""] + 1e-13
    assert err["+crt+last"] <= 2 * err["+last"] + 1e-13
    assert err["+i8x6"] <= max(1e-9, 2 * err[""])
    assert err["+i8x4"] <= 1e-5
    if base != "f16_scaled":
        assert err["+last"] <= 2 * err[""] + 1e-13


@pytest.mark.parametrize("n", [64, 300, 513])
def test_int8_residual_tiles_and_tails(ns, handle, n):
    """Padded n = 256, 512, 768: one to nine int8 tiles with ragged tails;
    radix-15 (contraction-aware table) in split-BF16 with the int8 residual
    equals the FP64-residual form to FP64 rounding of the residual."""
    w = workloads.symmetric(n, 0.9, 30 + n)
    k = 3375
    ref = series.radix15c(w.A, k)[0]
    f64, _, _ = run(ns, handle, w.A, k, "radix15c", "split_bf16")
    i8, rep, _ = run(ns, handle, w.A, k, "radix15c", "split_bf16+i8")
    crt, rep2, _ = run(ns, handle, w.A, k, "radix15c", "split_bf16+crt")
    assert rep["n_internal"] % 256 == 0 and rep2["n_internal"] == rep["n_internal"]
    e64 = assert_close(f64, ref, BAR["split_bf16"], "fp64 residual")[0]
    e8 = assert_close(i8, ref, BAR["split_bf16"], "int8 residual")[0]
    ec = assert_close(crt, ref, BAR["split_bf16"], "residue-form residual")[0]
    assert e8 <= 2 * e64 + 1e-13
    assert ec <= 2 * e64 + 1e-13


def test_int8_residual_hensel_nonsymmetric(ns, handle):
    """Hensel lifting (every product a residual step's) on a nonsymmetric
    input, FP32 products with the int8 residual, against the oracle."""
    g = workloads.gaussian(300, 0.8, 17)
    ref = series.hensel(g.A, 64)[0]
    for dt in ("f32_acc64+i8", "f32_acc64+crt"):
        got, rep, _ = run(ns, handle, g.A, 64, "hensel", dt)
        assert_close(got, ref, BAR["f32_acc64"], f"hensel {dt}")
        assert not rep["nonfinite"]


def test_residual_modifier_errors(ns, handle):
    """Modifiers apply only to residual methods in the FP64-accumulating
    forms; slice counts above 8 or without the int8 flag are refused.  Every
    case is rejected on the host before anything is enqueued."""
    A = torch.eye(64, dtype=torch.float64, device="cuda") * 0.5
    bad = [("radix9", "split_bf16+last", -2), ("radix9_resid", "f64+i8", -2),
           ("binary", "f16_scaled+i8", -2), ("radix9_resid", ns.SPLIT_BF16 | ns.RESID_INT8(9), -1),
           ("radix9_resid", ns.SPLIT_BF16 | (3 << 12), -1), ("radix9_resid", ns.SPLIT_BF16 | 0x800, -1),
           ("radix9", "split_bf16+crt", -2), ("radix9_resid", "f64+crt", -2),
           ("radix9_resid", ns.SPLIT_BF16 | ns.RESID_INT8(0) | ns.RESID_CRT, -1)]
    for method, dtype, status in bad:
        with pytest.raises(ns.NSError) as ei:
            ns.ns_eval_ex(A, 81, method, dtype, handle=handle)
        assert ei.value.status == status, (method, dtype)
    # a valid call still runs afterwards
    out = ns.ns_eval_ex(A, 81, "radix9_resid", "split_bf16+i8", handle=handle)
    torch.cuda.synchronize()
    lam = 0.5
    np.testing.assert_allclose(out.diag().cpu().numpy(), (1 - lam ** 81) / (1 - lam), rtol=1e-12)


@pytest.mark.parametrize("mod", ["+i8", "+crt"])
def test_emulated_residual_edge_inputs(ns, handle, mod):
    """A = 0 gives S = I exactly (every row and column maximum is zero, so
    every digit or residue is zero); a NaN in A is reported through the
    nonfinite flag (its row's maximum is not finite, so the emulated
    product writes NaN there), not raised."""
    n = 200
    got, rep, _ = run(ns, handle, np.zeros((n, n)), 81, "radix9_resid", "split_bf16" + mod)
    assert np.array_equal(got, np.eye(n)) and not rep["nonfinite"]
    A = workloads.symmetric(n, 0.7, 9).A.copy()
    A[7, 11] = np.nan
    _, rep, _ = run(ns, handle, A, 81, "radix9_resid", "split_bf16" + mod)
    assert rep["nonfinite"]
