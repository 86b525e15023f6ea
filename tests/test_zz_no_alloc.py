"""ns_eval_noalloc (the entry point that allocates nothing) against ns_eval_ex.

Both run the same schedule and kernels, so for every case the no-allocation
result must equal the handle path's bit for bit (and hence meet the parity
tolerance of its dtype against the oracle, which the handle path's own tests
show).  Each case makes two calls in a row on the library's fixed device
array, the second with a smaller matrix, so the second call runs on what the
first left there.  Run by name on a GPU:

    python -m pytest tests/test_zz_no_alloc.py -m gpu
"""

import sys

import numpy as np
import pytest

import workloads
from oracle import series

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32_acc64": 1e-5, "split_bf16": 1e-4, "f16_scaled": 1e-2,
       "split_bf16+i8": 1e-4}

# (method, dtype, first n, second n, k): both tile families of the small sizes,
# ragged tails, the mixed forms with their FP64 copies and max-abs slots
CASES = [
    ("radix9", "f64", 300, 150, 81),
    ("binary", "f32", 256, 100, 729),
    ("radix9_resid", "split_bf16", 200, 64, 81),
    ("radix9", "f16_scaled", 300, 37, 81),
    ("radix15c", "f64", 300, 129, 3375),
    ("mixed", "f32_acc64", 129, 65, 100),
    ("radix9_resid", "split_bf16+i8", 300, 64, 729),
]


@pytest.fixture(scope="module")
def ns():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_11843_amd as ns
    return ns


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(A, dtype):
    t = torch.from_numpy(np.ascontiguousarray(A))
    return (t.to(torch.float32) if dtype == "f32" else t.to(torch.float64)).cuda()


@pytest.mark.parametrize("method,dtype,n1,n2,k", CASES)
def test_noalloc_matches_handle_path(ns, method, dtype, n1, n2, k):
    h = ns.Handle(torch.cuda.current_device())
    try:
        for n, seed in ((n1, 11), (n2, 12)):
            w = workloads.symmetric(n, 0.9, seed)
            A = to_dev(w.A, dtype)
            say(f"[gpu] noalloc {method} {dtype} n={n} k={k}")
            got, rep = ns.ns_eval_noalloc(A, k, method, dtype, report=True)
            ref, rep_ref = ns.ns_eval_ex(A, k, method, dtype, handle=h, report=True)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (method, dtype, n)
            assert rep["gemms_performed"] == rep_ref["gemms_performed"]
            # the level norms are sums of per-workgroup atomics, whose order
            # varies from run to run: equal to rounding
            np.testing.assert_allclose(rep["level_norm"], rep_ref["level_norm"], rtol=1e-12)
            assert not rep["nonfinite"]
            # and the handle path's tolerance against the oracle's definition
            k_eff = rep["k_eff"]
            Ain = w.A.astype(np.float32).astype(np.float64) if dtype == "f32" else w.A
            exact = series.closed_form(Ain, k_eff) if method != "radix15c" else \
                series.radix15c(Ain, k)[0]
            err = series.rel_fro(got.double().cpu().numpy(), exact)
            say(f"    bit-identical to ns_eval_ex; rel err {err:.3e} (tol {TOL[dtype]:g})")
            assert err < TOL[dtype]
    finally:
        h.close()


def test_noalloc_rejects_what_does_not_fit(ns):
    # n = 2048 in FP64 radix-9 needs about 300 MB: refused on the host, before
    # anything is enqueued
    A = torch.zeros((2048, 2048), dtype=torch.float64, device="cuda")
    with pytest.raises(ns.NSError) as ei:
        ns.ns_eval_noalloc(A, 81, "radix9", "f64")
    assert ei.value.status == -5
    assert "fixed region" in str(ei.value)
    # and a call that fits still runs afterwards
    w = workloads.symmetric(64, 0.5, 3)
    A = to_dev(w.A, "f64")
    got = ns.ns_eval_noalloc(A, 81, "radix9", "f64")
    ref = ns.ns_eval_ex(A, 81, "radix9", "f64")
    torch.cuda.synchronize()
    assert torch.equal(got, ref)


def test_noalloc_back_to_back_calls_keep_their_own_parameters(ns):
    """Two calls in a row on one stream with no synchronisation between them:
    the second call's parameter upload must not reach the array before the
    first call's kernels have read it (the upload is ordered on the stream),
    so both results equal the handle path's."""
    w1 = workloads.symmetric(300, 0.9, 21)
    w2 = workloads.symmetric(150, 0.5, 22)
    A1, A2 = to_dev(w1.A, "f64"), to_dev(w2.A, "f64")
    o1 = torch.empty_like(A1)
    o2 = torch.empty_like(A2)
    ns.ns_eval_noalloc(A1, 729, "radix9", "f64", out=o1)
    ns.ns_eval_noalloc(A2, 81, "binary", "f64", out=o2)
    torch.cuda.synchronize()
    assert torch.equal(o1, ns.ns_eval_ex(A1, 729, "radix9", "f64"))
    assert torch.equal(o2, ns.ns_eval_ex(A2, 81, "binary", "f64"))
