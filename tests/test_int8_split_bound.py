"""The error model of the int8-slice emulation of an FP64 product
(NS_RESID_INT8 in ns.h), checked on the host with exact integer arithmetic.

The emulation cuts X by rows and Y by columns into s signed 7-bit digits under
a power of two per row / column and keeps the digit products with p + q <=
s + 1.  ns.h states an error of about n 2^(e_i + f_j) (s + 1) 2^(-7 s); the GPU
tests of the residual forms rely on it for their tolerances.  This model is
test code written from that description (it shares nothing with the HIP
kernels): digits, the int32 range of one diagonal's sum, and the bound against
the exact product.
"""

from fractions import Fraction

import numpy as np
import pytest


def split(M, s, axis):
    """(exponents, digit planes): M = 2^e (sum_p D_p 2^-7p + r 2^-7s)."""
    mx = np.max(np.abs(M), axis=axis, keepdims=True)
    e = np.where(mx > 0, np.frexp(mx)[1], 0)          # mx < 2^e
    x = np.ldexp(M, -e)
    planes = []
    for _ in range(s):
        t = x * 128.0
        d = np.trunc(t)
        x = t - d
        planes.append(d.astype(np.int64))
    return e, planes


def emulate(X, Y, s):
    ex, D = split(X, s, axis=1)
    fy, E = split(Y, s, axis=0)
    acc = np.zeros((X.shape[0], Y.shape[1]))
    worst = 0
    for d in range(s + 1, 1, -1):
        Cd = sum(D[p - 1] @ E[d - p - 1] for p in range(1, d))
        worst = max(worst, int(np.abs(Cd).max()))
        acc = acc + Cd.astype(np.float64) * 2.0 ** (-7 * d)
    return np.ldexp(acc, ex + fy), ex, fy, D, worst


def exact_product(X, Y):
    Xf = [[Fraction(float(v)) for v in row] for row in X]
    Yf = [[Fraction(float(v)) for v in row] for row in Y]
    n, k, m = X.shape[0], X.shape[1], Y.shape[1]
    return [[sum(Xf[i][t] * Yf[t][j] for t in range(k)) for j in range(m)] for i in range(n)]


def inputs(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n)) * np.exp2(rng.integers(-20, 20, (n, 1)))   # row scales
    Y = rng.standard_normal((n, n)) * np.exp2(rng.integers(-20, 20, (1, n)))   # column scales
    X[0, :] = 0.0                                                              # a zero row
    X[1, 3] = 2.0 ** -60                                                       # a tiny entry
    return X, Y


@pytest.mark.parametrize("s", [1, 2, 4, 7, 8])
def test_digits_reconstruct_within_one_unit(s):
    X, _ = inputs(40, s)
    e, D = split(X, s, axis=1)
    for P in D:
        assert P.min() >= -127 and P.max() <= 127
    rec = sum(P.astype(np.float64) * 2.0 ** (-7 * (p + 1)) for p, P in enumerate(D))
    # the remainder after s digits is below one unit of the last digit
    assert np.all(np.abs(np.ldexp(X, -e) - rec) < 2.0 ** (-7 * s))


@pytest.mark.parametrize("s", [3, 5, 7, 8])
def test_emulated_product_within_stated_bound(s):
    n = 24
    X, Y = inputs(n, 100 + s)
    got, ex, fy, _, worst = emulate(X, Y, s)
    assert worst * 1.0 <= (s) * n * 127 ** 2 < 2 ** 31       # one diagonal's int32 sum
    ref = exact_product(X, Y)
    bound = n * np.ldexp(np.ones((n, n)), ex + fy) * (s + 1) * 2.0 ** (-7 * s)
    err = np.array([[abs(float(Fraction(float(got[i, j])) - ref[i][j])) for j in range(n)]
                    for i in range(n)])
    assert np.all(err <= bound), float(np.max(err / bound))
    # and the bound is not vacuous: with one diagonal fewer the error exceeds it
    if s >= 3:
        short, *_ = emulate(X, Y, s - 2)
        err2 = np.array([[abs(float(Fraction(float(short[i, j])) - ref[i][j])) for j in range(n)]
                         for i in range(n)])
        assert np.any(err2 > bound)
