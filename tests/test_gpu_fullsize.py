"""GPU parity at the full n = 8192 workload sizes, in the launch configuration
bench.py times.

- precision_sym (symmetric, lam ~ U[-0.9, 0.9], k = 729): every output element
  against the spectral definition Q diag((1 - lam^k)/(1 - lam)) Q^T (one
  n^3 host product).
- gaussian_rho (nonsymmetric, rho_hat 0.99, k = 3375): sampled columns of the
  closed form (I - A)^{-1} (I - A^k) from an FP64 LU factorisation, with A^k E
  formed by repeated squaring (A^4096 is still ~1e-9 in norm here: the
  power-iteration estimate sits slightly below the true spectral radius).
  The FP32 legs are compared with the closed form for the FP32-rounded A that
  the GPU receives, so that the input's rounding (amplified by the
  conditioning of I - A) is not charged to the kernels.
"""

import sys

import numpy as np
import pytest

import workloads
from conftest import assert_close
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
    say("[cpu] generating precision_sym n=8192 and its spectral definition at k=729")
    w = workloads.make("precision_sym")
    return w, series.spectral_form(w.Q, w.lam, 729)


@pytest.mark.parametrize("method,dtype,tol", [
    ("radix9", "f64", 1e-12),
    ("radix9", "f32", 1e-5),
    ("radix9", "f32_acc64", 1e-5),
    ("radix9", "split_bf16", 1e-4),
    ("radix9", "f16_scaled", 1e-2),
    ("radix9_resid", "split_bf16", 1e-8),
    ("radix9_resid", "f16_scaled", 1e-6),
    # the residual-product variants (measured 7.8e-11, 7.6e-11, 3.8e-10)
    ("radix9_resid", "split_bf16+last", 1e-8),
    ("radix9_resid", "split_bf16+i8", 1e-8),
    ("radix9_resid", "split_bf16+i8x6", 1e-8),
])
def test_precision_workload(ns, precision_input, method, dtype, tol):
    w, ref = precision_input
    A = torch.from_numpy(w.A).cuda()
    if dtype == "f32":
        A = A.float()
    say(f"[gpu] precision_sym {method} {dtype} n=8192 k=729")
    out, rep = ns.ns_eval_ex(A, 729, method, dtype, report=True)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    del out, A
    assert rep["gemms_performed"] == 15 and not rep["nonfinite"] and rep["k_eff"] == 729
    # FP32: the reference is the FP64 definition for the unrounded A; with
    # lam <= 0.9 the input's rounding contributes at most ~2^-24 / (1 - 0.9)
    assert_close(got, ref, tol, f"{method} {dtype}")


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
    for rho, ks in ((0.99, (3375, 4096, 6561)), (0.95, (3375, 4096))):
        A = g.A * (rho / 0.99)
        say(f"[cpu] closed-form reference rho={rho}: A^k E by squaring, LU of I - A")
        AkE = powers_times(A, E, ks)
        for prec in ("f64", "f32"):
            # the FP32 path receives A rounded to FP32: its reference is the
            # closed form for that matrix.  A^k E is taken from the unrounded A
            # for both: the rounding changes it by about k 2^-24 ||A^k||, below
            # 1e-12 of the result, far under the FP32 bar
            Ap = A if prec == "f64" else A.astype(np.float32).astype(np.float64)
            lu = scipy.linalg.lu_factor(np.eye(8192) - Ap)
            for k in ks:
                refs[(prec, rho, k)] = scipy.linalg.lu_solve(lu, E - AkE[k])
            refs[(prec, rho, None)] = scipy.linalg.lu_solve(lu, E)          # (I - A)^{-1}
            del lu, Ap
        del A
    return g, cols, refs


# All-FP32 schedules on the rho_hat = 0.99 input do not meet the FP32 bar of
# 1e-5.  I - A has kappa_2 = 2.3e3 (||(I - A)^{-1}||_2 = 909), so one FP32
# rounding of an iterate already moves the result by up to kappa 2^-24 =
# 1.4e-4; measured against the closed form for the FP32-rounded A: binary
# 1.1e-5, radix-15 (contraction-aware table) 1.5e-5, any-k 1.7e-5, radix-9
# 3.4e-5.  The same kernels meet 1e-12 in FP64 on this input, and the
# residual forms with FP32 products and an FP64 residual (f32_acc64) meet the
# FP32 bar; those legs follow.
FP32_BELOW_BAR = pytest.mark.xfail(
    strict=True, reason="all-FP32 storage on kappa(I - A) = 2.3e3: 1.1e-5 to 3.4e-5, above 1e-5")


@pytest.mark.parametrize("method,dtype,rho,tol,k", [
    ("radix9", "f64", 0.99, 1e-12, 3375),
    ("binary", "f64", 0.99, 1e-12, 3375),
    pytest.param("radix9", "f32", 0.99, 1e-5, 3375, marks=FP32_BELOW_BAR),
    pytest.param("binary", "f32", 0.99, 1e-5, 3375, marks=FP32_BELOW_BAR),
    pytest.param("mixed", "f32", 0.99, 1e-5, 3375, marks=FP32_BELOW_BAR),
    pytest.param("radix15c", "f32", 0.99, 1e-5, 3375, marks=FP32_BELOW_BAR),
    # FP32 products, FP64 running sum and FP64 residual: the residual
    # iteration corrects the FP32 products' errors
    ("radix15c", "f32_acc64", 0.99, 1e-5, 3375),
    ("radix9_resid", "f32_acc64", 0.99, 1e-5, 3375),
    ("hensel", "f32_acc64", 0.99, 1e-5, 3375),
    ("radix15", "f32", 0.95, 1e-5, 3375),
    ("radix15", "f64", 0.95, 1e-12, 3375),
    # the contraction-aware table converges at rho 0.99 as well.  In FP64 one
    # more level is used: at t = 3 the residual E^[3](A) is still ~6e-9 in
    # Frobenius norm on this nonnormal matrix (R_2 has norm 1.6 though its
    # spectral radius is below 0.1), so Y_3 differs from (I - A)^{-1} by ~1e-9
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
    say(f"   level norms {['%.3g' % x for x in rep['level_norm']]}")
    # only the all-FP32 path receives a rounded A; the others read it in FP64
    prec = "f32" if dtype == "f32" else "f64"
    assert_close(got, refs[(prec, rho, k_ref)], tol, f"{method} {dtype} rho={rho} (sampled columns)")
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
