"""GPU parity of the batched form (one persistent launch, cached HIP graph)
against the oracle and against the per-matrix launch loop."""

import json
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


def pack(mats):
    offs = np.zeros(len(mats), dtype=np.int64)
    total = 0
    for i, M in enumerate(mats):
        offs[i] = total
        total += M.size
    buf = np.zeros(total, dtype=np.float32)
    for i, M in enumerate(mats):
        buf[offs[i]:offs[i] + M.size] = M.astype(np.float32).ravel()
    return buf, offs


def unpack(buf, offs, ns_):
    return [buf[o:o + n * n].reshape(n, n) for o, n in zip(offs, ns_)]


def device_batch(mats):
    buf, offs = pack(mats)
    ns_ = np.array([M.shape[0] for M in mats], dtype=np.int32)
    return (torch.from_numpy(buf).cuda(), torch.from_numpy(offs).cuda(),
            torch.from_numpy(ns_).cuda(), torch.from_numpy(ns_), offs, ns_)


def mixed_batch(seed=0):
    rng = np.random.default_rng(seed)
    sizes = [1, 8, 13, 16, 32, 50, 64, 65, 100, 128, 129, 200, 256] * 3
    rng.shuffle(sizes)
    return [workloads.jacobi(int(n), rng) for n in sizes]


@pytest.mark.parametrize("method", ["radix9", "binary", "naive"])
def test_batched_matches_oracle(ns, method):
    mats = mixed_batch(1)
    A, offd, nd, nh, offs, ns_ = device_batch(mats)
    k = 20 if method == "naive" else 81
    say(f"[gpu] batched {method} batch={len(mats)} k={k}")
    out, rep = ns.ns_eval_batched(A, offd, nd, nh, k, method, "f32", report=True)
    torch.cuda.synchronize()
    got = unpack(out.cpu().numpy(), offs, ns_)
    worst = 0.0
    for M, G in zip(mats, got):
        ref, _ = series.evaluate(M.astype(np.float32).astype(np.float64), k, method)
        worst = max(worst, series.rel_fro(G, ref))
    say(f"   worst rel err {worst:.3e}")
    assert worst < 1e-5
    assert not rep["nonfinite"]
    assert rep["gemms_performed"] == ns.ns_plan(k, method)[2]


@pytest.mark.parametrize("method", ["binary", "naive"])
def test_batched_exact_on_signed_cycles(ns, method):
    """Every matrix a scaled signed n-cycle (workloads.cyclic): at k = 16 each
    entry of every operand and product is a sum of signed powers 2^-j,
    j <= 16, so the FP32 batched kernel is exact and must equal S_16 in every
    element, for every n the tile shapes meet (n = 1 .. 3 wrap the cycle
    around, which keeps the sums within 17 bits)."""
    rng = np.random.default_rng(5)
    sizes = [1, 2, 3, 8, 13, 16, 32, 50, 64, 65, 100, 128, 129, 200, 255, 256] * 2
    rng.shuffle(sizes)
    mats = [workloads.cyclic(int(n), 900 + i) for i, n in enumerate(sizes)]
    A, offd, nd, nh, offs, ns_ = device_batch(mats)
    say(f"[gpu] batched exact signed cycles {method} batch={len(mats)} k=16")
    out = ns.ns_eval_batched(A, offd, nd, nh, 16, method, "f32")
    torch.cuda.synchronize()
    got = unpack(out.cpu().numpy(), offs, ns_)
    for M, G in zip(mats, got):
        ref = series.permutation_form(M, 16)
        assert np.array_equal(G.astype(np.float64), ref), (method, M.shape[0])


def test_batched_bit_identical_to_launch_loop(ns):
    """Same tile arithmetic, same padding: the persistent kernel and the
    per-matrix launch loop must agree bit for bit."""
    mats = mixed_batch(2)
    A, offd, nd, nh, offs, ns_ = device_batch(mats)
    say(f"[gpu] batched vs loop batch={len(mats)}")
    a = ns.ns_eval_batched(A, offd, nd, nh, 81, "radix9", "f32")
    b = ns.ns_eval_batched_loop(A, torch.from_numpy(offs), nh, 81, "radix9", "f32")
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_graph_replays_are_identical(ns):
    """The cached graph is replayed with unrelated device work and host
    synchronisation in between; every replay must equal the first result."""
    mats = mixed_batch(3)
    A, offd, nd, nh, offs, ns_ = device_batch(mats)
    h = ns.Handle(0)
    out = torch.empty_like(A)
    first = ns.ns_eval_batched(A, offd, nd, nh, 81, "radix9", "f32", out_packed=out, handle=h).clone()
    for i in range(4):
        x = torch.randn(512, 512, device="cuda")
        (x @ x).sum().item()                      # other work between replays
        out.zero_()
        ns.ns_eval_batched(A, offd, nd, nh, 81, "radix9", "f32", out_packed=out, handle=h)
        torch.cuda.synchronize()
        assert torch.equal(out, first), f"replay {i}"
    h.close()


def test_batched_k1_identity_and_empty(ns):
    mats = mixed_batch(4)[:10]
    A, offd, nd, nh, offs, ns_ = device_batch(mats)
    out = ns.ns_eval_batched(A, offd, nd, nh, 1, "radix9", "f32")
    torch.cuda.synchronize()
    for G, n in zip(unpack(out.cpu().numpy(), offs, ns_), ns_):
        assert np.array_equal(G, np.eye(n))
    empty = torch.zeros(1, device="cuda")
    z = torch.zeros(1, dtype=torch.int64, device="cuda")
    ns.ns_eval_batched(empty, z, z.int(), torch.zeros(0, dtype=torch.int32), 81, "radix9", "f32",
                       out_packed=empty)


def test_batched_rejects_unsupported(ns):
    mats = [np.eye(300) * 0.5]
    A, offd, nd, nh, offs, ns_ = device_batch(mats)
    with pytest.raises(ns.NSError) as e:
        ns.ns_eval_batched(A, offd, nd, nh, 81, "radix9", "f32")
    assert e.value.status == -2
    with pytest.raises(ns.NSError) as e:
        ns.ns_eval_batched(A, offd, nd, nh, 81, "radix15", "f32")
    assert e.value.status == -2


def test_binding_checks_packed_extents(ns):
    """Packed buffers that cannot hold the matrices, or offsets of the wrong
    type, are refused before any launch."""
    mats = mixed_batch(12)[:4]
    A, offd, nd, nh, offs, ns_ = device_batch(mats)
    short = A[: A.numel() - 1]
    with pytest.raises(ValueError):
        ns.ns_eval_batched(short, offd, nd, nh, 81, "radix9", "f32")
    with pytest.raises(TypeError):
        ns.ns_eval_batched(A, offd.int(), nd, nh, 81, "radix9", "f32")
    with pytest.raises(ValueError):
        ns.ns_eval_batched(A, offd, nd, nh, 81, "radix9", "f32", out_packed=torch.empty_like(short))
    bad = torch.from_numpy(offs).clone()
    bad[-1] += 1                                   # last matrix now ends past the buffer
    with pytest.raises(ValueError):
        ns.ns_eval_batched_loop(A, bad, nh, 81, "radix9", "f32")


def test_autotune_then_evaluate(ns, tmp_path, monkeypatch):
    monkeypatch.setenv("NS_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    mats = mixed_batch(5)
    A, offd, nd, nh, offs, ns_ = device_batch(mats)
    h = ns.Handle(0)
    out = torch.empty_like(A)
    say("[gpu] autotune")
    n_timed = ns.ns_autotune_batched(A, offd, nd, nh, 81, out, handle=h)
    assert n_timed >= 1
    got = ns.ns_eval_batched(A, offd, nd, nh, 81, "radix9", "f32", out_packed=out, handle=h)
    ref = ns.ns_eval_batched_loop(A, torch.from_numpy(offs), nh, 81, "radix9", "f32", handle=h)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    assert (tmp_path / "tune.jsonl").read_text().count("\"big\"") == 1
    h.close()


def test_graph_cache_after_workspace_growth_and_eviction(ns, tmp_path, monkeypatch):
    """One handle evaluates a small batch, then makes calls that grow its
    workspace (the autotuner on a larger batch, then a larger batch still),
    then uses more distinct buffer sets than its graph cache holds.  Every
    repeat of the small batch must equal its first result: graphs captured
    against an older workspace are captured again, never replayed."""
    monkeypatch.setenv("NS_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    h = ns.Handle(0)
    small = device_batch(mixed_batch(7)[:3])
    large = device_batch(mixed_batch(8))
    larger = device_batch(mixed_batch(9) + mixed_batch(10))

    def run(b, out):
        A, offd, nd, nh = b[:4]
        return ns.ns_eval_batched(A, offd, nd, nh, 81, "radix9", "f32", out_packed=out, handle=h)

    out_s = torch.empty_like(small[0])
    first = run(small, out_s).clone()
    torch.cuda.synchronize()

    def check(tag):
        out_s.zero_()
        run(small, out_s)
        torch.cuda.synchronize()
        assert torch.equal(out_s, first), tag

    say(f"[gpu] graph cache: autotuner on batch={len(large[4])}")
    A, offd, nd, nh = large[:4]
    ns.ns_autotune_batched(A, offd, nd, nh, 81, torch.empty_like(A), handle=h)
    check("after autotuning a larger batch")
    say(f"[gpu] graph cache: batch={len(larger[4])}")
    run(larger, torch.empty_like(larger[0]))
    check("after a larger batch")
    say("[gpu] graph cache: 20 more buffer sets")
    keep = []                      # distinct buffers, so that each call has its own graph
    for i in range(20):
        b = device_batch(mixed_batch(11 + i)[:2])
        keep.append(b)
        run(b, torch.empty_like(b[0]))
    check("after eviction")
    h.close()


def hist_key(ns_):
    """The batched path's key for a batch's n histogram (ascending n)."""
    vals, counts = np.unique(ns_, return_counts=True)
    return "".join(f"{v}:{c}," for v, c in zip(vals, counts))


# tile configurations of the persistent kernel: 128x128, 64x128, 128x64, and
# 128x128 with 128x256 direct-to-LDS tiles for n > 128
@pytest.mark.parametrize("big", [0, 1, 2, 3])
def test_every_tile_config(ns, tmp_path, monkeypatch, big):
    """Each configuration the autotuner may pick, forced through the tuning
    file: bit-identical to the per-matrix launch loop and within FP32
    rounding of the oracle, for every method."""
    mats = mixed_batch(6)
    A, offd, nd, nh, offs, ns_ = device_batch(mats)
    path = tmp_path / "tune.jsonl"
    path.write_text(json.dumps({"hist": hist_key(ns_), "big": big, "per_cu": 2}) + "\n")
    monkeypatch.setenv("NS_TUNE_CACHE", str(path))
    h = ns.Handle(0)
    for method, k in (("radix9", 81), ("binary", 81), ("naive", 12)):
        say(f"[gpu] batched tile config {big} {method} batch={len(mats)}")
        got = ns.ns_eval_batched(A, offd, nd, nh, k, method, "f32", handle=h)
        ref = ns.ns_eval_batched_loop(A, torch.from_numpy(offs), nh, k, method, "f32", handle=h)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), method
        worst = 0.0
        for M, G in zip(mats, unpack(got.cpu().numpy(), offs, ns_)):
            o, _ = series.evaluate(M.astype(np.float32).astype(np.float64), k, method)
            worst = max(worst, series.rel_fro(G, o))
        assert worst < 1e-5, (method, worst)
    h.close()


@pytest.mark.slow
def test_jacobi_batch_workload(ns):
    """The 2048-matrix workload in full against the oracle, matrix by matrix."""
    w = workloads.make("jacobi_batch")
    A, offd, nd, nh, offs, ns_ = device_batch(w.mats)
    say(f"[gpu] jacobi_batch batch={len(w.mats)}")
    out, rep = ns.ns_eval_batched(A, offd, nd, nh, 81, "radix9", "f32", report=True)
    torch.cuda.synchronize()
    got = unpack(out.cpu().numpy(), offs, ns_)
    worst = 0.0
    for M, G in zip(w.mats, got):
        ref, _ = series.radix9(M.astype(np.float32).astype(np.float64), 81)
        worst = max(worst, series.rel_fro(G, ref))
    say(f"   worst rel err {worst:.3e}")
    assert worst < 1e-5


def test_batched_reads_n_only_from_the_host_array(ns):
    """The kernel takes each matrix's n from the library's own copy of n_host
    (uploaded with the work queue); the device array n_dev is not read, so a
    call without one gives the same bits."""
    mats = mixed_batch(6)
    A, offd, nd, nh, offs, ns_ = device_batch(mats)
    h = ns.Handle(0)
    a = ns.ns_eval_batched(A, offd, nd, nh, 81, "radix9", "f32", handle=h).clone()
    b = ns.ns_eval_batched(A, offd, None, nh, 81, "radix9", "f32", handle=h)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    h.close()


def test_graph_cache_keys_on_each_matrix_n(ns):
    """Two calls on the same buffers with the same histogram of n but the
    sizes in a different order: the second must not replay the first call's
    queue.  (The buffers are sized for either assignment, so even a stale
    queue would stay inside them.)"""
    rng = np.random.default_rng(9)
    m8, m16 = workloads.jacobi(8, rng), workloads.jacobi(16, rng)
    A = torch.zeros(2 * 16 * 16, dtype=torch.float32, device="cuda")
    out = torch.zeros_like(A)
    offd = torch.zeros(2, dtype=torch.int64, device="cuda")
    h = ns.Handle(0)
    for order in ((m8, m16), (m16, m8)):
        buf, offs = pack(order)
        A.zero_()
        A[:buf.size] = torch.from_numpy(buf).cuda()
        offd.copy_(torch.from_numpy(offs))
        nh = torch.tensor([M.shape[0] for M in order], dtype=torch.int32)
        ns.ns_eval_batched(A, offd, None, nh, 81, "radix9", "f32", out_packed=out, handle=h)
        torch.cuda.synchronize()
        got = unpack(out.cpu().numpy(), offs, nh.numpy())
        for M, G in zip(order, got):
            ref, _ = series.radix9(M.astype(np.float32).astype(np.float64), 81)
            assert series.rel_fro(G, ref) < 1e-5
    h.close()
