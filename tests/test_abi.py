"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/ns.h declares, and its host-only logic (planning,
product counts, radix-15 table, status strings, argument errors) agrees with
the oracle and the paper."""

import ctypes
import os
import re

import pytest

from conftest import ROOT, golden_rows
from oracle import coeffs15, series

LIB = os.path.join(ROOT, "paper_2602_11843_amd", "libns.so")


@pytest.fixture(scope="module")
def ns():
    if not os.path.exists(LIB):
        from paper_2602_11843_amd import build
        build.build()
    import paper_2602_11843_amd as ns
    return ns


def _declared_functions():
    with open(os.path.join(ROOT, "include", "ns.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(ns_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("ns_eval", "ns_eval_ex", "ns_eval_batched", "ns_plan", "ns_create",
                     "ns_destroy", "ns_status_string", "ns_workspace_bytes"):
        assert required in names


def test_library_exports_every_declared_symbol(ns):
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_abi(ns):
    for name in _declared_functions():
        if name in ("ns_create", "ns_destroy", "ns_last_error"):
            continue
        if name in ("ns_set_product_timing", "ns_product_timing", "ns_product_timing_dtype",
                    "ns_product_timing_launches"):
            assert hasattr(ns.Handle, name)
        else:
            assert hasattr(ns, name), name


METHOD_MAP = {"naive": "naive", "binary": "binary", "radix9": "radix9", "radix15": "radix15",
              "radix9_resid": "radix9_resid", "quinary": "quinary", "ternary": "ternary",
              "hensel": "hensel", "mixed": "mixed", "radix15c": "radix15c"}


@pytest.mark.parametrize("method", list(METHOD_MAP))
def test_plan_matches_oracle(ns, method):
    for k in (1, 2, 3, 8, 9, 10, 80, 81, 82, 125, 225, 729, 3375, 4096, 6561, 10 ** 6):
        assert ns.ns_plan(k, method) == series.plan(k, METHOD_MAP[method]), (method, k)


def test_plan_reproduces_table2(ns):
    cols = {"binary": 1, "quinary": 2, "radix9": 3, "radix15": 4}
    for row in golden_rows("table2_counts.txt"):
        for method, c in cols.items():
            if row[c] != "-":
                assert ns.ns_plan(int(row[0]), method)[2] == int(row[c])


def test_plan_errors(ns):
    with pytest.raises(ns.NSError) as e:
        ns.ns_plan(0, "radix9")
    assert e.value.status == -1
    with pytest.raises(ns.NSError) as e:
        ns.ns_plan(10, 99)
    assert e.value.status == -1
    with pytest.raises(ns.NSError) as e:           # k_eff = 15^17 overflows int64
        ns.ns_plan(2 ** 63 - 1, "radix15")
    assert e.value.status == -5


def test_radix15_table_agrees_with_oracle(ns):
    """The library derives its table with its own Gauss-Newton (C++, long
    double); it must land on the oracle's polished doubles."""
    c, pe, s15, s16 = ns.ns_radix15_coeffs()
    ref = coeffs15.polished()
    for a, b in zip(c, ref):
        assert abs(a - b) <= 4 * abs(b) * 2.0 ** -52
    assert pe < 1e-15
    assert round(s15, 3) == 0.185 and round(s16, 3) == 0.458


def test_radix15c_table_agrees_with_oracle(ns):
    """The contraction-aware table: the library polishes its own copy of the
    six-decimal start point; it must land on the oracle's polished doubles,
    with the error quadratic's coefficients 1 - a15, a15 - a16, a16 positive."""
    c, pe, s15, s16 = ns.ns_radix15c_coeffs()
    ref = coeffs15.contract_polished()
    for a, b in zip(c, ref):
        assert abs(a - b) <= 4 * abs(b) * 2.0 ** -52
    assert pe < 1e-15
    assert min(1 - s15, s15 - s16, s16) > 0.11


def test_workspace_bytes(ns):
    b9 = ns.ns_workspace_bytes(4096, "radix9", "f64")
    assert b9 >= 9 * 4096 * 4096 * 8
    assert ns.ns_workspace_bytes(4096, "radix9", "f32") < b9
    with pytest.raises(ns.NSError):
        ns.ns_workspace_bytes(0, "radix9", "f64")


def test_workspace_bytes_of_the_emulated_residuals(ns):
    """The emulated residual adds its planes to the workspace: s digit planes
    per operand and an FP64 partial-sum matrix for the digit form, one plane
    per modulus for each operand and for the reduced products in the residue
    form (ns.h: 14 moduli at n = 8192, 13 at n = 256)."""
    base = ns.ns_workspace_bytes(8192, "radix9_resid", "split_bf16")
    mat = 8192 * 8192
    i8 = ns.ns_workspace_bytes(8192, "radix9_resid", "split_bf16+i8") - base
    crt = ns.ns_workspace_bytes(8192, "radix9_resid", "split_bf16+crt") - base
    assert 2 * 7 * mat + 8 * mat <= i8 < 2 * 7 * mat + 8 * mat + 2 ** 20
    assert 3 * 14 * mat <= crt < 3 * 14 * mat + 2 ** 20
    small = ns.ns_workspace_bytes(200, "hensel", "f32_acc64+crt") - \
        ns.ns_workspace_bytes(200, "hensel", "f32_acc64")
    assert 3 * 13 * 256 * 256 <= small < 3 * 13 * 256 * 256 + 2 ** 20
    with pytest.raises(ns.NSError):                       # unknown modifier bits
        ns.ns_workspace_bytes(256, "radix9_resid", ns.SPLIT_BF16 | 0x800)


def test_status_strings(ns):
    assert ns.ns_status_string(0) == "ok"
    assert "argument" in ns.ns_status_string(-1)
    assert ns.ns_status_string(-4).startswith("HIP")


def test_mixed_plan_matches_oracle_for_every_k(ns):
    """The library's exact any-k planner (C++) and the oracle's (Python) are
    written separately; both must find the same product count and number of
    radix updates for every k up to 2000 and for large k."""
    ks = list(range(1, 2001)) + [3375, 4095, 4097, 10 ** 6, 10 ** 9 + 7, 2 ** 40 + 5, 2 ** 62 + 1]
    for k in ks:
        assert ns.ns_plan(k, "mixed") == series.plan(k, "mixed"), k


def test_binding_refuses_bad_tensors_before_the_library(ns):
    """Wrong element types and host tensors are refused by the binding
    itself, before any call into the library (none reaches the GPU)."""
    import torch
    A = torch.zeros((8, 8), dtype=torch.float64)
    with pytest.raises(TypeError):
        ns.ns_eval_ex(A.float(), 9, "radix9", "f64")            # FP64 I/O, FP32 tensor
    with pytest.raises(TypeError):
        ns.ns_eval_ex(A, 9, "radix9", "f32")                    # FP32 I/O, FP64 tensor
    with pytest.raises(ValueError):
        ns.ns_eval_ex(A, 9, "radix9", "f64")                    # host memory
    with pytest.raises(TypeError):
        ns.ns_eval(A.float(), 9, "radix9", "split_bf16")        # split forms take FP64
    buf = torch.zeros(64, dtype=torch.float32)
    n = torch.tensor([8], dtype=torch.int32)
    with pytest.raises(TypeError):
        ns.ns_eval_batched(buf, torch.zeros(1, dtype=torch.int32), n, n, 81)   # offsets are int64
    with pytest.raises(TypeError):
        ns.ns_eval_batched(buf.double(), torch.zeros(1, dtype=torch.int64), n, n, 81)
    with pytest.raises(ValueError):
        ns.ns_eval_batched_loop(buf, torch.zeros(1, dtype=torch.int64), n, 81)  # host memory


def test_radix15_tables_built_concurrently_match():
    """The two radix-15 tables are built on first use, each under its own
    once-flag; first uses from two host threads at the same time must give
    the tables a single thread gives.  A fresh process makes both calls the
    first ones."""
    import subprocess
    import sys
    code = r'''
import threading, sys
sys.path.insert(0, sys.argv[1])
import paper_2602_11843_amd as ns
out = {}
go = threading.Barrier(2)
def first(name, fn):
    go.wait()
    out[name] = fn()
ts = [threading.Thread(target=first, args=(nm, fn)) for nm, fn in
      (("b", ns.ns_radix15_coeffs), ("c", ns.ns_radix15c_coeffs))]
for t in ts: t.start()
for t in ts: t.join()
print(repr(out["b"][0]))
print(repr(out["c"][0]))
'''
    res = subprocess.run([sys.executable, "-c", code, ROOT], capture_output=True, text=True,
                         timeout=300)
    assert res.returncode == 0, res.stderr
    got_b, got_c = (eval(line) for line in res.stdout.strip().splitlines())
    for got, ref in ((got_b, coeffs15.polished()), (got_c, coeffs15.contract_polished())):
        for a, b in zip(got, ref):
            assert abs(a - b) <= 4 * abs(b) * 2.0 ** -52
