"""Pins of the oracle's per-level norms (host only).

Every radix schedule of the oracle reports one Frobenius norm per level: for
the telescoping schedules (Sec. 2.2) the power A^(m^l) that the next level
uses, for the general iteration of eq. (8) (Sec. 5.3) the residual R_l.  Both
have closed forms that run no matrix schedule:

- for A = Q diag(lam) Q^T with Q orthogonal (Q = I for a diagonal A),
  ||A^N||_F = sqrt(sum_i lam_i^(2N)), the Frobenius norm being invariant under
  orthogonal similarity;
- for the general iteration R_l = E^[l](A) (Lemma 5.9), so on a diagonal A the
  residual is diag(E^[l](lam_i)), E^[l] the l-fold composition of the scalar
  error map E(z) = 1 - (1 - z) f(z) (Definition 5.2) of the kernel polynomial.

Diagonal inputs are exact rationals, so both sides are exact until the final
conversion of the sum of squares to a double.  The last tests plant an
off-by-one-level mistake (the norm taken before the level's update) in a copy
of a schedule and show that the pin rejects it.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import coeffs15, poly, series

LAM = [Fraction(1, 2), Fraction(-3, 5), Fraction(9, 10)]


def diag_matrix(lam):
    n = len(lam)
    A = np.empty((n, n), dtype=object)
    A[:, :] = Fraction(0)
    for i, v in enumerate(lam):
        A[i, i] = v
    return A


def power_norm(lam, N):
    """||diag(lam)^N||_F from the eigenvalues."""
    return math.sqrt(float(sum(x ** (2 * N) for x in lam)))


def residual_norm(lam, E, levels):
    """||diag(E^[levels](lam))||_F: the error map applied `levels` times to
    each eigenvalue, exactly."""
    vals = list(lam)
    for _ in range(levels):
        vals = [poly.evaluate(E, v) for v in vals]
    return math.sqrt(float(sum(v * v for v in vals)))


def norms_match(got, want, rtol=1e-13):
    return len(got) == len(want) and all(
        abs(g - w) <= rtol * abs(w) for g, w in zip(got, want))


TELESCOPING = {"binary": (2, 64), "ternary": (3, 81), "quinary": (5, 125), "radix9": (9, 729)}


@pytest.mark.parametrize("method", list(TELESCOPING))
def test_telescoping_norms_are_the_powers_exactly(method):
    """Level l reports ||A^(m^(l+1))||_F (ns_report's definition)."""
    m, k = TELESCOPING[method]
    _, rep = series.evaluate(diag_matrix(LAM), k, method)
    want = [power_norm(LAM, m ** (l + 1)) for l in range(rep["levels"])]
    assert norms_match(rep["level_norms"], want), (rep["level_norms"], want)


@pytest.mark.parametrize("method", list(TELESCOPING))
def test_telescoping_norms_on_a_dense_symmetric_matrix(method):
    """The same identity on a dense float64 A = Q diag(lam) Q^T, with one
    eigenvalue near 1 so that every level's power stays well above the
    rounding of the schedule."""
    m, k = TELESCOPING[method]
    rng = np.random.default_rng(77)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    lam = rng.uniform(-0.9, 0.9, 40)
    lam[0] = 0.995
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    _, rep = series.evaluate(A, k, method)
    want = [math.sqrt(float(np.sum(lam ** (2 * m ** (l + 1))))) for l in range(rep["levels"])]
    assert np.allclose(rep["level_norms"], want, rtol=1e-9, atol=0)


def test_mixed_norms_follow_the_plan():
    """The exact any-k schedule reports the power after each radix update; the
    exponent after each step follows its plan (radix m: n -> m n; additive
    step: n -> n + 1)."""
    k = 1000
    _, steps = series.mixed_plan(k)
    n, want = 1, []
    for m in steps:
        if m == 1:
            n += 1
        else:
            n *= m
            want.append(power_norm(LAM, n))
    _, rep = series.mixed(diag_matrix(LAM), k)
    assert norms_match(rep["level_norms"], want)


RESIDUAL = {
    "radix9_resid": (lambda: poly.radix9_poly(), 81),
    "quinary_resid": (lambda: poly.quinary_poly(), 125),
    "hensel": (lambda: poly.hensel_poly(), 16),
    "radix15": (lambda: poly.radix15_poly(coeffs15.polished()), 225),
    "radix15c": (lambda: poly.radix15_poly(coeffs15.contract_polished()), 225),
}


@pytest.mark.parametrize("method", list(RESIDUAL))
def test_residual_norms_are_the_error_map_iterates(method):
    """Level l reports ||R_(l+1)||_F = ||E^[l+1](A)||_F (Lemma 5.9)."""
    f_of, k = RESIDUAL[method]
    E = poly.error_map(f_of())
    _, rep = series.evaluate(diag_matrix(LAM), k, method)
    want = [residual_norm(LAM, E, l + 1) for l in range(rep["levels"])]
    assert norms_match(rep["level_norms"], want), (rep["level_norms"], want)


def test_exact_kernel_error_maps_are_pure_powers():
    """For the exact kernels E(z) = z^m, so the residual pin above reduces to
    the power pin: an independent route to the same numbers."""
    for f, m in ((poly.radix9_poly(), 9), (poly.quinary_poly(), 5), (poly.hensel_poly(), 2)):
        assert poly.error_map(f) == poly.z_pow(m)


# --- planted mistakes ---------------------------------------------------------

def _telescoping_norm_before_update(A, k, method, kernel):
    """A copy of the telescoping schedule with one mistake: the level's norm
    is taken of the power it started from, not of the new one."""
    k_eff, t, _ = series.plan(k, method)
    mm = series._Counter()
    I = series._eye(A)
    S, P = I.copy(), A.copy()
    norms = []
    for _ in range(t):
        T = kernel(P, mm)
        S = mm(S, T)
        norms.append(series._fro(P))                      # planted: before the update
        P = I - T + mm(T, P)
    return S, {"levels": t, "level_norms": norms}


def _general_norm_before_update(A, k, method, kernel):
    """A copy of the general iteration with the same mistake."""
    k_eff, t, _ = series.plan(k, method)
    mm = series._Counter()
    I = series._eye(A)
    M = I - A
    Y, R = I.copy(), A.copy()
    norms = []
    for _ in range(t):
        Y = mm(Y, kernel(R, mm))
        norms.append(series._fro(R))                      # planted: the old residual
        R = I - mm(M, Y)
    return Y, {"levels": t, "level_norms": norms}


def test_planted_off_by_one_level_fails_the_power_pin():
    _, rep = _telescoping_norm_before_update(diag_matrix(LAM), 729, "radix9", series.kernel_radix9)
    want = [power_norm(LAM, 9 ** (l + 1)) for l in range(rep["levels"])]
    assert not norms_match(rep["level_norms"], want)
    # the correct schedule passes the same check
    _, good = series.radix9(diag_matrix(LAM), 729)
    assert norms_match(good["level_norms"], want)


def test_planted_off_by_one_level_fails_the_residual_pin():
    c28 = coeffs15.polished()
    kern = lambda B, mm: series.kernel_radix15(B, mm, c28)  # noqa: E731
    _, rep = _general_norm_before_update(diag_matrix(LAM), 225, "radix15", kern)
    E = poly.error_map(poly.radix15_poly(c28))
    want = [residual_norm(LAM, E, l + 1) for l in range(rep["levels"])]
    assert not norms_match(rep["level_norms"], want)
