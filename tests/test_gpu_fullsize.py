"""GPU parity at the full n = 8192 workload sizes, in the launch configuration
bench.py times, on sampled outputs the CPU can compute one by one.

- precision_sym (symmetric, lam ~ U[-0.9, 0.9], k = 729): sampled columns of the
  spectral definition Q diag((1 - lam^k)/(1 - lam)) Q^T.
- gaussian_rho (nonsymmetric, rho_hat 0.99, k = 3375): sampled columns of the
  closed form (I - A)^{-1} (I - A^k) from an FP64 LU factorisation, with A^k E
  formed by repeated squaring (A^4096 is still ~1e-9 in norm here: the
  power-iteration estimate sits slightly below the true spectral radius).
"""

import sys

import numpy as np
import pytest

import workloads
from oracle import series

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]


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
def precision_input():
    say("[cpu] generating precision_sym n=8192")
    return workloads.make("precision_sym")


@pytest.mark.parametrize("method,dtype,tol", [
    ("radix9", "f64", 1e-12),
    ("radix9", "f32", 1e-5),
    ("radix9", "f32_acc64", 1e-5),
    ("radix9", "split_bf16", 1e-4),
    ("radix9", "f16_scaled", 1e-2),
    ("radix9_resid", "split_bf16", 1e-8),
    ("radix9_resid", "f16_scaled", 1e-6),
])
def test_precision_workload(ns, precision_input, method, dtype, tol):
    w = precision_input
    A = torch.from_numpy(w.A).cuda()
    if dtype == "f32":
        A = A.float()
    say(f"[gpu] precision_sym {method} {dtype} n=8192 k=729")
    out, rep = ns.ns_eval_ex(A, 729, method, dtype, report=True)
    torch.cuda.synchronize()
    cols = np.sort(np.random.default_rng(1).choice(8192, 24, replace=False))
    got = out[:, torch.from_numpy(cols).cuda()].double().cpu().numpy()
    ref = series.spectral_form(w.Q, w.lam, rep["k_eff"], cols=cols)
    err = series.rel_fro(got, ref)
    say(f"   sampled rel err {err:.3e}")
    assert err < tol
    assert rep["gemms_performed"] == 15 and not rep["nonfinite"]


def powers_times(A, E, ks):
    """{k: A^k E} for the given k by repeated squaring of A (k < 2^13)."""
    out = {k: E.copy() for k in ks}
    P = A.copy()
    for j in range(13):
        for k in ks:
            if (k >> j) & 1:
                out[k] = P @ out[k]
        if j < 12:
            P = P @ P
    return out


@pytest.fixture(scope="module")
def gaussian_input():
    import scipy.linalg
    say("[cpu] generating gaussian_rho n=8192 (400 power iterations)")
    g = workloads.make("gaussian_rho")
    cols = np.sort(np.random.default_rng(2).choice(8192, 12, replace=False))
    E = np.zeros((8192, len(cols)))
    E[cols, np.arange(len(cols))] = 1.0
    refs = {}
    for rho, ks in ((0.99, (4096, 6561)), (0.95, (3375, 4096))):
        A = g.A * (rho / 0.99)
        say(f"[cpu] closed-form reference rho={rho}: A^k E by squaring, LU of I - A")
        AkE = powers_times(A, E, ks)
        lu = scipy.linalg.lu_factor(np.eye(8192) - A)
        for k in ks:
            refs[(rho, k)] = scipy.linalg.lu_solve(lu, E - AkE[k])
        refs[(rho, None)] = scipy.linalg.lu_solve(lu, E)          # (I - A)^{-1}
        del lu, A
    return g, cols, refs


@pytest.mark.parametrize("method,dtype,rho,tol,k", [
    ("radix9", "f64", 0.99, 1e-12, 3375),
    ("binary", "f64", 0.99, 1e-12, 3375),
    # FP32 on this nonnormal, rho ~ 0.99 input: the powers grow transiently
    # (||A^9||_F ~ 79) before decaying, and FP32 rounding is amplified by the
    # conditioning of I - A; the measured errors are 9e-6 (binary) and 4e-5
    # (radix-9), both far below the conditioning bound kappa * 2^-24
    ("radix9", "f32", 0.99, 1e-4, 3375),
    ("binary", "f32", 0.99, 1e-4, 3375),
    ("radix15", "f32", 0.95, 1e-5, 3375),
    ("radix15", "f64", 0.95, 1e-12, 3375),
    # the contraction-aware table converges at rho 0.99 as well.  In FP64 one
    # more level is used: at t = 3 the residual E^[3](A) is still ~6e-9 in
    # Frobenius norm on this nonnormal matrix (R_2 has norm 1.6 though its
    # spectral radius is below 0.1), so Y_3 differs from (I - A)^{-1} by ~1e-9
    ("radix15c", "f32", 0.99, 1e-4, 3375),
    ("radix15c", "f64", 0.99, 1e-12, 15 ** 4),
])
def test_gaussian_workload(ns, gaussian_input, method, dtype, rho, tol, k):
    g, cols, refs = gaussian_input
    A = torch.from_numpy(g.A * (rho / 0.99)).cuda()
    if dtype == "f32":
        A = A.float()
    say(f"[gpu] gaussian_rho rho={rho} {method} {dtype} n=8192 k={k}")
    out, rep = ns.ns_eval_ex(A, k, method, dtype, report=True)
    torch.cuda.synchronize()
    got = out[:, torch.from_numpy(cols).cuda()].double().cpu().numpy()
    # radix-15 is the residual iteration: Y_t = (I - E^[t](A)) (I - A)^{-1}
    # (Lemma 5.9), which at rho 0.95 and t = 3 equals S_k to far below 1e-12;
    # with the contraction-aware table at rho 0.99, E^[3](A) is the final
    # residual (level norm ~1e-13), so Y_3 is compared with (I - A)^{-1}
    k_ref = {"radix15": 3375, "radix15c": None}.get(method, rep["k_eff"])
    err = series.rel_fro(got, refs[(rho, k_ref)])
    say(f"   sampled rel err vs closed form {err:.3e}; level norms {['%.3g' % x for x in rep['level_norm']]}")
    assert err < tol
    # the last level's norm (power or residual) is far below the first; an FP32
    # residual recomputed as I - Y + A Y stops at its rounding floor (~1e-3 in
    # Frobenius norm at n = 8192 with this conditioning)
    assert rep["level_norm"][-1] < 1e-3 * rep["level_norm"][0]


def test_radix15_divergence_is_reported_at_rho_099(ns, gaussian_input):
    """rho_hat = 0.99 lies outside the basin of the radix-15 error map
    E(z) = z^15 (c + d z + e z^2) (|z| up to about 0.97): the iteration
    diverges, which the report shows as growing level norms, not as an error."""
    g, cols, refs = gaussian_input
    A = torch.from_numpy(g.A).float().cuda()
    out, rep = ns.ns_eval_ex(A, 3375, "radix15", "f32", report=True)
    torch.cuda.synchronize()
    ln = rep["level_norm"]
    say(f"   radix15 rho 0.99 level norms {['%.3g' % x for x in ln]}")
    assert ln[-1] > ln[0] > 1.0
