"""Bit-for-bit parity of every exact schedule, at its real length, on inputs
where floating-point arithmetic is exact.

``workloads.cyclic`` gives A = diag(s) P / 2 for one random signed n-cycle P:
A^j (j < n) is a signed permutation times 2^-j whose nonzeros sit where no
other power's do.  Every operand the exact schedules form (sums of distinct
powers with small integer weights) and every product of two of them then has
one term per output element, a signed power of two times a small integer, so
the FP64, FP32, split-BF16, scaled-FP16 and int8-slice products are all exact
and each kernel must reproduce S_k(A) in every element.  Unlike the k = 4
inputs of ``test_gpu_exact_dyadic.py``, this runs ternary (k = 27), quinary
(k = 25), Hensel (k = 32), binary splitting (k = 32) and the any-k schedule
(k = 75 = 3 * 5 * 5 and k = 30 = 2 * 3 * 5, no radix-9 step) over all their
levels.  The radix-9 kernel of Theorem 3.1 is left out: its weights (3/20,
11/40, 767/800) are not dyadic, so its products round.

Range limits of the scaled-FP16 form: operands span 1 .. 2^-j and are scaled
so their max lies in [2^14, 2^15), which keeps every scaled value a normal
FP16 number while j <= 28.  The widest operand of the FP16 cases is the
any-k schedule's T_5(A^6) at k = 30, with A^24 beside I (k = 75 would put
A^60 beside I in one operand).  The int8 residual is exact while a column
of Y needs at most 7 s bits (Hensel at k = 32 needs 16).

References: the oracle at n = 300; the closed form ``series.permutation_form``
(pinned to exact rationals and to the oracle in ``test_dyadic_exact.py``) at
the panel, large-tile and full (n = 8192) sizes, where the oracle's FP64
products would take the test past a minute.
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


ALL = ["f64", "f32", "f32_acc64", "split_bf16", "f16_scaled"]
# (method, k for FP64/FP32/split-BF16, k for scaled FP16, dtypes)
SCHEDULES = [
    ("binary", 32, 32, ALL),
    ("naive", 16, 16, ["f64", "f32"]),        # no FP64-accumulated Horner form
    ("hensel", 32, 32, ALL),
    ("ternary", 27, 27, ALL),
    ("quinary", 25, 25, ALL),
    ("mixed", 75, 30, ALL),
]

_A = {}


def cyc(n):
    if n not in _A:
        _A[n] = workloads.cyclic(n, 700 + n)
    return _A[n]


def run(ns, A, k, method, dtype):
    Ad = torch.from_numpy(A.astype(np.float32) if dtype == "f32" else A).cuda()
    out, rep = ns.ns_eval_ex(Ad, k, method, dtype, report=True)
    torch.cuda.synchronize()
    assert not rep["nonfinite"] and rep["k_eff"] == k, (method, dtype, rep["k_eff"])
    return out.cpu().numpy().astype(np.float64), rep


def check(got, ref, *what):
    bad = int(np.count_nonzero(got != ref))
    assert bad == 0, (*what, bad, float(np.max(np.abs(got - ref))))


@pytest.mark.parametrize("method,k,k16,dtypes", SCHEDULES, ids=[s[0] for s in SCHEDULES])
def test_small_tiles_equal_oracle(ns, method, k, k16, dtypes):
    A = cyc(300)
    refs = {}
    for dtype in dtypes:
        kk = k16 if dtype == "f16_scaled" else k
        if kk not in refs:
            refs[kk], _ = series.evaluate(A, kk, method)
            assert np.array_equal(refs[kk], series.permutation_form(A, kk))
        say(f"[gpu] exact cyclic {method} k={kk} {dtype} n=300")
        got, _ = run(ns, A, kk, method, dtype)
        check(got, refs[kk], method, dtype, kk)


# padded sizes of the 16-bit panel paths
PANEL = {(2600, "f16_scaled"): 2816, (3072, "f16_scaled"): 3072, (3072, "split_bf16"): 3072}


@pytest.mark.parametrize("n", [2600, 3072, 4096])
@pytest.mark.parametrize("method,k,k16,dtypes", [s for s in SCHEDULES if s[0] != "naive"],
                         ids=[s[0] for s in SCHEDULES if s[0] != "naive"])
def test_large_tiles_equal_closed_form(ns, n, method, k, k16, dtypes):
    A = cyc(n)
    refs = {}
    for dtype in dtypes:
        kk = k16 if dtype == "f16_scaled" else k
        if kk not in refs:
            refs[kk] = series.permutation_form(A, kk)
        say(f"[gpu] exact cyclic {method} k={kk} {dtype} n={n}")
        got, rep = run(ns, A, kk, method, dtype)
        check(got, refs[kk], method, dtype, kk, n)
        if (n, dtype) in PANEL:
            assert rep["n_internal"] == PANEL[(n, dtype)]


@pytest.mark.parametrize("method,k,k16", [("binary", 64, 32), ("ternary", 27, 27)])
def test_full_size_exact(ns, method, k, k16):
    """n = 8192, the size of the precision-form and large FP32 workloads: every
    engine in the launch configuration those workloads time (FP64 128 x 128
    and FP32 128 x 256 tiles, both 16-bit panel products), bit for bit."""
    n = 8192
    A = cyc(n)
    refs = {}
    for dtype in ALL:
        kk = k16 if dtype == "f16_scaled" else k
        if kk not in refs:
            refs[kk] = series.permutation_form(A, kk)
        say(f"[gpu] exact cyclic {method} k={kk} {dtype} n={n}")
        got, rep = run(ns, A, kk, method, dtype)
        check(got, refs[kk], method, dtype, kk, n)
        assert rep["n_internal"] == n
        del got


@pytest.mark.parametrize("n", [300, 3072, 8192])
@pytest.mark.parametrize("dtype", ["f32_acc64+i8", "split_bf16+i8+last", "f16_scaled+i8x6",
                                   "split_bf16+crt", "f16_scaled+crt+last"])
def test_int8_residual_exact_cyclic(ns, n, dtype):
    """Hensel at k = 32 with the emulated residual: A's rows need one digit
    and Y's columns (S_16) three, within the s + 1 digit-pair bound; in the
    residue form both fit 46-bit integers exactly."""
    A = cyc(n)
    say(f"[gpu] exact cyclic hensel k=32 {dtype} n={n}")
    got, rep = run(ns, A, 32, "hensel", dtype)
    check(got, series.permutation_form(A, 32), dtype, n)
    # the final residual is A^32 exactly: a signed permutation times 2^-32
    assert rep["level_norm"][-1] == pytest.approx(np.sqrt(n) * 2.0 ** -32, rel=1e-15)
