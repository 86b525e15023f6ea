"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Inputs are the seeded workloads (``workloads``); for the FP32 path the oracle
receives the same FP32-rounded matrix in float64, so the comparison measures
the kernels' arithmetic only.  Tolerances (relative Frobenius error):
FP64 1e-12, FP32 1e-5.
"""

import sys

import numpy as np
import pytest

import workloads
from conftest import assert_close
from oracle import series

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32_acc64": 1e-5, "split_bf16": 1e-4}


@pytest.fixture(scope="module")
def ns():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_11843_amd as ns
    return ns


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(A, dtype):
    t = torch.from_numpy(np.ascontiguousarray(A))
    t = t.to(torch.float32) if dtype == "f32" else t.to(torch.float64)
    return t.cuda()


def oracle_input(A, dtype):
    """What the GPU actually receives, in float64 for the oracle."""
    return A.astype(np.float32).astype(np.float64) if dtype == "f32" else A


def run(ns, A, k, method, dtype, **kw):
    say(f"[gpu] {method} {dtype} n={A.shape[0]} k={k}")
    out, rep = ns.ns_eval_ex(dev(A, dtype), k, method, dtype, report=True, **kw)
    torch.cuda.synchronize()
    return out.double().cpu().numpy(), rep


ORACLE_NAME = {"naive": "naive", "binary": "binary", "radix9": "radix9", "radix15": "radix15",
               "radix9_resid": "radix9_resid", "quinary": "quinary", "ternary": "ternary",
               "hensel": "hensel", "radix15c": "radix15c"}


# --- small sizes: every method x {f64, f32}, several tiles and ragged tails ---

@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("method", ["naive", "binary", "radix9", "radix15", "radix9_resid",
                                    "quinary", "ternary", "hensel", "radix15c"])
@pytest.mark.parametrize("n", [37, 256, 300])
def test_small_parity(ns, method, dtype, n):
    w = workloads.symmetric(n, 0.9, 100 + n)
    k = 20 if method == "naive" else 81
    got, rep = run(ns, w.A, k, method, dtype)
    ref, orep = series.evaluate(oracle_input(w.A, dtype), k, ORACLE_NAME[method])
    assert_close(got, ref, TOL[dtype], f"{method} {dtype} n={n}")
    assert rep["k_eff"] == orep["k_eff"]
    assert rep["gemms_performed"] == rep["gemms_formula"] == orep["products"]
    assert not rep["nonfinite"]
    if method != "naive":
        # per-level norms; in FP32 a residual recomputed as I - Y + A Y cannot go
        # below the FP32 rounding floor (~ n * 2^-24), so small norms are
        # compared absolutely
        ln, on = np.array(rep["level_norm"]), np.array(orep["level_norms"])
        if dtype == "f32":
            assert np.allclose(ln, on, rtol=1e-3, atol=n * 2.0 ** -22)
        else:
            assert np.allclose(ln, on, rtol=1e-9, atol=1e-12)


# FP64 products at padded n in [160, 256] use the split-K 16 x 16 tile: its
# lower edge (150 -> 160), ragged tails (200 -> 224, 225 -> 256) and a
# non-symmetric input, every epilogue shape the schedules use
@pytest.mark.parametrize("method", ["naive", "binary", "radix9", "radix15c", "radix9_resid", "ternary"])
@pytest.mark.parametrize("n", [150, 200, 225])
def test_splitk_range_parity(ns, method, n):
    w = workloads.gaussian(n, 0.9, 300 + n) if n == 225 else workloads.symmetric(n, 0.9, 300 + n)
    k = 20 if method == "naive" else 81
    got, rep = run(ns, w.A, k, method, "f64")
    ref, orep = series.evaluate(w.A, k, ORACLE_NAME[method])
    say(f"   n_internal {rep['n_internal']}")
    assert rep["n_internal"] in (160, 224, 256)
    assert_close(got, ref, TOL["f64"], f"{method} n={n}")
    assert not rep["nonfinite"]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("method", ["binary", "radix9", "radix15", "radix15c"])
def test_nonsymmetric_parity(ns, method, dtype):
    g = workloads.gaussian(512, 0.95, 7)
    k = 225 if method == "radix15" else 81
    got, _ = run(ns, g.A, k, method, dtype)
    ref, _ = series.evaluate(oracle_input(g.A, dtype), k, method)
    assert_close(got, ref, TOL[dtype], f"{method} {dtype} nonsymmetric")


# --- the n = 256, k = 81 workload in full --------------------------------------

@pytest.mark.parametrize("method", ["naive", "binary", "radix9"])
def test_small_symmetric_workload(ns, method):
    w = workloads.make("small_symmetric")
    got, rep = run(ns, w.A, 81, method, "f64")
    # critical path in launches: binary's S (I + P) and P P share a launch at
    # this size (7 levels), as do radix-9's sum and power updates (4 per level)
    assert rep["product_launches"] == {"naive": 80, "binary": 7, "radix9": 8}[method]
    ref, _ = series.evaluate(w.A, 81, method)
    closed = series.spectral_form(w.Q, w.lam, rep["k_eff"])
    assert_close(got, ref, 1e-12, f"{method} vs oracle")
    assert_close(got, closed, 1e-12, f"{method} vs closed form")


# --- edge cases -------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("method", ["naive", "binary", "radix9", "radix15", "hensel"])
def test_k1_is_identity(ns, method, dtype):
    w = workloads.symmetric(40, 0.5, 3)
    got, rep = run(ns, w.A, 1, method, dtype)
    assert rep["gemms_performed"] == 0 and rep["k_eff"] == 1
    assert np.array_equal(got, np.eye(40))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_n1(ns, dtype):
    A = np.array([[0.5]])
    got, rep = run(ns, A, 81, "radix9", dtype)
    assert abs(got[0, 0] - (1 - 0.5 ** 81) / 0.5) < 1e-14 * (1 if dtype == "f64" else 1e8)


def test_leading_dimension(ns):
    w = workloads.symmetric(100, 0.8, 4)
    big = torch.zeros((100, 128), dtype=torch.float64, device="cuda")
    big[:, :100] = dev(w.A, "f64")
    out = torch.full((100, 160), 7.0, dtype=torch.float64, device="cuda")
    ns.ns_eval_ex(big[:, :100], 81, "radix9", "f64", out=out[:, :100])
    torch.cuda.synchronize()
    ref, _ = series.radix9(w.A, 81)
    assert_close(out[:, :100].cpu().numpy(), ref, 1e-12, "lda/ldo > n")
    assert torch.all(out[:, 100:] == 7.0)          # nothing written past ldo's n columns


def test_short_form_matches_full_form(ns):
    w = workloads.symmetric(64, 0.7, 5)
    A = dev(w.A, "f64")
    a = ns.ns_eval(A, 81, "radix9", "f64")
    b = ns.ns_eval_ex(A, 81, "radix9", "f64")
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_nonfinite_is_reported_not_raised(ns):
    A = workloads.symmetric(64, 0.7, 6).A.copy()
    A[3, 5] = np.nan
    got, rep = run(ns, A, 81, "radix9", "f64")
    assert rep["nonfinite"]


def test_divergence_is_reported(ns):
    """rho > 1 is the caller's problem: the growth shows in the level norms."""
    A = 1.2 * np.eye(32)
    got, rep = run(ns, A, 81, "radix9", "f64")
    assert rep["level_norm"][-1] > rep["level_norm"][0] > 1


def test_argument_errors(ns):
    A = dev(np.eye(8) * 0.5, "f64")
    with pytest.raises(ns.NSError) as e:
        ns.ns_eval_ex(A, 0, "radix9", "f64")
    assert e.value.status == -1
    with pytest.raises(ns.NSError) as e:
        ns.ns_eval_ex(A, 9, "radix9", "f64", out=A)        # out overlaps A
    assert e.value.status == -1
    with pytest.raises(ns.NSError) as e:
        ns.ns_eval_ex(A, 9, "naive", "split_bf16")
    assert e.value.status == -2
    empty = torch.zeros((0, 0), dtype=torch.float64, device="cuda")
    with pytest.raises(ns.NSError) as e:
        ns.ns_eval_ex(empty, 9, "radix9", "f64", out=torch.zeros((0, 0), dtype=torch.float64,
                                                                  device="cuda"))
    assert e.value.status == -1
    # n above the supported range is refused before any memory is touched: both
    # matrices are views of one short row (row stride 0), never read
    n = 65537
    row = torch.zeros(n, dtype=torch.float64, device="cuda")
    other = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(ns.NSError) as e:
        ns.ns_eval_ex(row.as_strided((n, n), (0, 1)), 9, "radix9", "f64",
                      out=other.as_strided((n, n), (0, 1)))
    assert e.value.status == -5


def test_repeat_calls_are_deterministic(ns):
    w = workloads.symmetric(300, 0.9, 8)
    a, _ = run(ns, w.A, 729, "radix9", "f64")
    b, _ = run(ns, w.A, 729, "radix9", "f64")
    assert np.array_equal(a, b)


def test_threads_share_the_default_handles(ns):
    """Host threads calling the short form (the library's default handle)
    and the full form without a handle (the binding's default handle) at the
    same time: every result equals the one computed alone."""
    import threading
    sizes = (96, 130, 200, 300)
    A = [dev(workloads.symmetric(n, 0.8, 20 + i).A, "f64") for i, n in enumerate(sizes)]
    ref_short = [ns.ns_eval(a, 81, "radix9", "f64") for a in A]
    ref_full = [ns.ns_eval_ex(a, 81, "radix9", "f64") for a in A]
    torch.cuda.synchronize()
    errors = []

    def work(i):
        try:
            for r in range(5):
                s = ns.ns_eval(A[i], 81, "radix9", "f64")
                f = ns.ns_eval_ex(A[i], 81, "radix9", "f64")
                torch.cuda.synchronize()
                if not (torch.equal(s, ref_short[i]) and torch.equal(f, ref_full[i])):
                    errors.append((sizes[i], r))
        except Exception as e:          # reported below, in the main thread
            errors.append((sizes[i], repr(e)))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(A))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors


# --- large sizes: sampled outputs against the definition --------------------

@pytest.mark.slow
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_element_offsets_past_2_31(ns, dtype):
    """n = 46400 (padded to 46592 or 46464): element offsets past 2^31 in every product
    kernel's loads and stores.  Binary splitting at k = 2 on a diagonal A is
    S = I + A exactly (each product entry has one nonzero term), so entries
    sampled over the whole matrix, the last rows and columns included, are
    compared bit for bit."""
    n = 46400
    tdt = torch.float32 if dtype == "f32" else torch.float64
    g = torch.Generator(device="cuda").manual_seed(4640)
    d = (torch.rand(n, device="cuda", generator=g, dtype=torch.float64) - 0.5).to(tdt)
    A = torch.zeros(n, n, device="cuda", dtype=tdt)
    A.diagonal().copy_(d)
    h = ns.Handle(0)
    say(f"[gpu] offsets past 2^31: binary k=2 {dtype} n={n}")
    out, rep = ns.ns_eval_ex(A, 2, "binary", dtype, handle=h, report=True)
    torch.cuda.synchronize()
    del A
    rng = np.random.default_rng(46400)
    rows = np.concatenate([rng.integers(0, n, 200), np.arange(n - 40, n)])
    cols = np.concatenate([rng.integers(0, n, 200), np.arange(n - 40, n)])
    ri, ci = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    got_diag = out[ri, ri].cpu()
    want_diag = (1 + d[ri]).cpu()
    assert torch.equal(got_diag, want_diag)
    off = rows != cols
    got_off = out[ri[torch.from_numpy(off).cuda()], ci[torch.from_numpy(off).cuda()]].cpu()
    assert torch.count_nonzero(got_off) == 0
    assert rep["n_internal"] == (46592 if dtype == "f32" else 46464) and not rep["nonfinite"]
    del out
    h.close()
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def large_symmetric():
    say("[cpu] generating large_symmetric n=4096")
    return workloads.make("large_symmetric")


@pytest.mark.slow
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("method", ["binary", "radix9"])
def test_large_symmetric_full(ns, large_symmetric, method, dtype):
    """n = 4096, k = 729 (large tiles of both engines): every output element
    against the oracle's own schedule on the input the GPU receives, and
    (FP64) against the spectral definition."""
    w = large_symmetric
    got, rep = run(ns, w.A, 729, method, dtype)
    say("[cpu] oracle schedule at n=4096")
    ref, orep = series.evaluate(oracle_input(w.A, dtype), 729, method)
    assert rep["gemms_performed"] == orep["products"]
    assert_close(got, ref, TOL[dtype], f"{method} {dtype} vs oracle")
    if dtype == "f64":
        assert_close(got, series.spectral_form(w.Q, w.lam, rep["k_eff"]), TOL[dtype],
                     "vs spectral definition")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [2100, 3000])
def test_mid_sizes_full(ns, n, dtype):
    """Sizes between the small and the large tiles (FP32 keeps its small tile
    up to 4096, FP64 switches at 2048), with a ragged tail: the whole result
    against the spectral closed form."""
    w = workloads.symmetric(n, 0.9, 40 + n)
    got, rep = run(ns, w.A, 81, "radix9", dtype)
    say(f"   n_internal {rep['n_internal']}")
    ref = series.spectral_form(w.Q, w.lam, rep["k_eff"])
    # FP32: the reference is the FP64 definition for the unrounded A, so the
    # input's rounding to FP32 is part of the error here (lam <= 0.9 keeps
    # its amplification to ~1/(1 - 0.9))
    assert_close(got, ref, TOL[dtype], f"radix9 {dtype} n={n}")


# --- exact S_k for any k (no round-up) ---------------------------------------

MIXED_KS = [1, 2, 3, 4, 5, 7, 10, 16, 27, 100, 128, 1000, 3375, 4097]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [37, 300])
def test_mixed_any_k_parity(ns, dtype, n):
    """Every plan shape: additive chains (k <= 5), fused final additive steps
    after each radix (k = 10, 16, 1000, 4097), radix 2, 3, 5 and 9 updates.
    Nonsymmetric input, so an operand-order mistake in the additive step
    (B A instead of A B is harmless, but S B instead of B S is not) fails."""
    g = workloads.gaussian(n, 0.6, 400 + n)
    for k in MIXED_KS:
        got, rep = run(ns, g.A, k, "mixed", dtype)
        ref, orep = series.mixed(oracle_input(g.A, dtype), k)
        say(f"   k={k} products {rep['gemms_performed']}")
        assert_close(got, ref, TOL[dtype], f"mixed {dtype} k={k}")
        assert rep["k_eff"] == k
        assert rep["gemms_performed"] == rep["gemms_formula"] == orep["products"]
        assert rep["levels"] == orep["levels"]
        ln, on = np.array(rep["level_norm"][:rep["levels"]]), np.array(orep["level_norms"])
        if dtype == "f32":
            assert np.allclose(ln, on, rtol=1e-3, atol=n * 2.0 ** -22)
        else:
            assert np.allclose(ln, on, rtol=1e-9, atol=1e-12)


def test_mixed_matches_closed_form_at_k_not_a_power(ns):
    w = workloads.symmetric(256, 0.95, 21)
    for k in (1000, 3375, 5000):
        got, rep = run(ns, w.A, k, "mixed", "f64")
        closed = series.spectral_form(w.Q, w.lam, k)
        assert rep["k_eff"] == k
        assert_close(got, closed, 1e-12, f"mixed k={k} vs closed form")


def test_product_timing_records_every_launch(ns):
    """Per-launch timing: one record per product launch of each call, in
    order, engines named by dtype; their sum equals the aggregate, and the
    launches of a call group into its levels (radix-9 at n = 2048, FP64: five
    products per level in four launches, the independent sum and power
    updates sharing one grid)."""
    w = workloads.symmetric(2048, 0.9, 5)
    A = torch.from_numpy(w.A).cuda()
    h = ns.Handle(torch.cuda.current_device())
    try:
        h.ns_set_product_timing(True)
        h.ns_product_timing(reset=True)
        for _ in range(2):
            _, rep = ns.ns_eval_ex(A, 729, "radix9", "f64", handle=h, report=True)
        launches = h.ns_product_timing_launches()
        cnt, total, _ = h.ns_product_timing(reset=True)
        h.ns_set_product_timing(False)
    finally:
        h.close()
    assert rep["product_launches"] == 12 and rep["gemms_performed"] == 15
    assert len(launches) == cnt == 2 * rep["product_launches"]
    assert all(e == ns.F64 and ms > 0 for ms, e in launches)
    assert abs(sum(ms for ms, _ in launches) - total) < 1e-3 * total
    say(f"   per level (last call): {[round(sum(ms for ms, _ in launches[12 + 4 * i:16 + 4 * i]), 3) for i in range(3)]} ms")
