"""Pins of the exact-arithmetic premise behind the bit-for-bit GPU tests in
``test_gpu_exact_dyadic.py``.

On ``workloads.dyadic`` inputs (entries k/8, at most three per row and
column) the first few powers of A, and I + A, have at most a handful of
significant bits, so every product a short schedule performs is exact in
FP64 -- and, the operands fitting in 8 significant bits, in FP32, BF16 and
FP16 too.  The oracle's FP64 binary splitting, Horner and Hensel iteration at
k = 4 must then equal the exact rational S_4(A) = I + A + A^2 + A^3 entry for
entry; that is checked here against Fractions, independently of any float.
"""

from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import series


def exact_s4(A):
    n = A.shape[0]
    F = [[Fraction(float(v)) for v in row] for row in A]
    def mul(X, Y):
        return [[sum(X[i][t] * Y[t][j] for t in range(n) if X[i][t] and Y[t][j]) for j in range(n)]
                for i in range(n)]
    A2 = mul(F, F)
    A3 = mul(A2, F)
    return [[(1 if i == j else 0) + F[i][j] + A2[i][j] + A3[i][j] for j in range(n)] for i in range(n)]


def significant_bits(x):
    """Bits between the leading and trailing set bit of |x| (0 for 0)."""
    if x == 0:
        return 0
    m, _ = np.frexp(abs(x))
    bits = 0
    while m != 0:
        m = m * 2 - np.floor(m * 2)
        bits += 1
    return bits


def test_generator_grid_and_norm():
    A = workloads.dyadic(64, 3)
    assert np.all(A * 8 == np.round(A * 8))
    assert np.abs(A).sum(axis=1).max() <= 3 / 8 and np.abs(A).sum(axis=0).max() <= 3 / 8
    assert np.count_nonzero(A) >= 64


@pytest.mark.parametrize("method", ["binary", "naive", "hensel"])
def test_oracle_equals_exact_rational(method):
    A = workloads.dyadic(40, 11)
    ref = exact_s4(A)
    got, _ = series.evaluate(A, 4, method)
    assert all(Fraction(float(got[i][j])) == ref[i][j] for i in range(40) for j in range(40))


def test_operands_fit_in_eight_bits():
    """The operands of the k = 4 schedules (I + A, A, A^2, A^4) carry at most
    8 significant bits per entry: bf16 holds them exactly (its low split part
    is zero), and so do fp16 and fp32."""
    A = workloads.dyadic(300, 5)
    I = np.eye(300)
    A2 = A @ A
    for M in (I + A, A, A2, A2 @ A2):
        assert max(significant_bits(v) for v in M.ravel()) <= 8


def exact_sk_cyclic(A, k):
    """S_k(A) = sum_{j<k} A^j in Fractions for A = scale * signed n-cycle,
    composing the cycle exactly (no floating point)."""
    n = A.shape[0]
    col = [int(np.flatnonzero(A[i])[0]) for i in range(n)]
    val = [Fraction(float(A[i, col[i]])) for i in range(n)]
    S = [dict() for _ in range(n)]
    for i in range(n):
        pos, coef = i, Fraction(1)
        for _ in range(k):
            S[i][pos] = S[i].get(pos, Fraction(0)) + coef
            coef *= val[pos]
            pos = col[pos]
    return S


# the schedules with dyadic weights, at the lengths the bit-for-bit GPU tests
# use (the any-k plans for 30 and 75 take radices 2, 3 and 5 only).  Radix-15
# approximates T_15, and the radix-9 kernel's weights 3/20, 11/40 and 767/800
# round in binary, so neither is exact here.
CYCLIC_CASES = [("binary", 32), ("naive", 16), ("hensel", 32), ("ternary", 27), ("quinary", 25),
                ("mixed", 30), ("mixed", 75)]


def test_cyclic_mixed_plans_avoid_radix9():
    assert 9 not in series.mixed_plan(30)[1] and 9 not in series.mixed_plan(75)[1]


@pytest.mark.parametrize("method,k", CYCLIC_CASES)
def test_oracle_exact_on_cyclic_inputs(method, k):
    """On a scaled signed n-cycle the powers A^j (j < n) occupy disjoint
    positions, each entry a signed power of 1/2: the oracle's FP64 schedule
    must equal the exact S_k entry for entry (n = 96 > k)."""
    n = 96
    A = workloads.cyclic(n, 7)
    got, rep = series.evaluate(A, k, method)
    assert rep["k_eff"] == k
    S = exact_sk_cyclic(A, k)
    for i in range(n):
        for j in range(n):
            assert Fraction(float(got[i][j])) == S[i].get(j, 0), (method, i, j)


@pytest.mark.parametrize("n,k", [(64, 40), (5, 16), (1, 9)])
def test_permutation_form_is_exact(n, k):
    """series.permutation_form, the reference of the GPU tests at the large
    sizes, equals the Fraction composition -- also for cycles shorter than k,
    where powers wrap onto earlier positions."""
    A = workloads.cyclic(n, 9)
    S = exact_sk_cyclic(A, k)
    ref = series.permutation_form(A, k)
    assert all(Fraction(float(ref[i, j])) == S[i].get(j, 0) for i in range(n) for j in range(n))


def test_permutation_form_matches_brute_force_on_general_rows():
    """One nonzero per row but not a permutation (two rows may point at one
    column): the row walk still equals explicit powers."""
    rng = np.random.default_rng(4)
    n = 12
    A = np.zeros((n, n))
    A[np.arange(n), rng.integers(0, n, n)] = rng.choice([-0.5, 0.25, 0.75], n)
    assert np.allclose(series.permutation_form(A, 7), series.brute_force(A, 7), rtol=0, atol=1e-15)
    with pytest.raises(ValueError):
        series.permutation_form(np.ones((3, 3)), 4)


def test_cyclic_powers_are_single_bits():
    A = workloads.cyclic(200, 3)
    P = np.eye(200)
    for j in range(1, 30):
        P = P @ A
        nz = P[P != 0]
        assert nz.size == 200 and np.all(np.abs(nz) == 0.5 ** j)
