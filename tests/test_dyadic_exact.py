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
