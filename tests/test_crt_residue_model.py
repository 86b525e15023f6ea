"""The residue form of the emulated FP64 product (NS_RESID_CRT in ns.h),
checked on the host.

ns.h states the scheme: rows of X and columns of Y scaled by powers of two to
integers X', Y' of at most 46 bits, residues modulo pairwise-coprime moduli
m <= 256 in the symmetric int8 range, one exact int32 product per modulus, and
the integer X'Y' rebuilt by the Chinese remainder theorem in FP64 limbs of 32
bits; N = 13 moduli at padded n = 256 and 14 from 512 to 65536.  This model is
test code written from that description (it shares nothing with the HIP
kernels).  It checks that

- the moduli are pairwise coprime and their product leaves X'Y' inside a
  quarter of M at every n the counts cover (so the nearest multiple of M is
  the right one),
- every residue fits int8 and every per-modulus sum fits int32,
- the FP64 limb arithmetic rebuilds X'Y' exactly (against Python integers),
- the result is within n 2^(e_i + f_j - 46) of the exact product.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

B = 46
MODULI = [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197, 193]
TWO32 = 2.0 ** 32


def count(n):
    """Moduli for padded n: their product exceeds n 2^(2B + 2)."""
    M = 1
    for l, m in enumerate(MODULI):
        M *= m
        if M > n << (2 * B + 2):
            return l + 1
    raise ValueError(n)


def scale(M, axis):
    mx = np.max(np.abs(M), axis=axis, keepdims=True)
    e = np.where(mx > 0, np.frexp(mx)[1], 0)          # mx < 2^e
    return e, np.rint(np.ldexp(np.ldexp(M, -e), B))   # |X'| <= 2^B, integers in float64


def residue8(x, m):
    """Symmetric int8 residue, as FP64 floor / fma would compute it."""
    q = np.floor(x * (1.0 / m))
    r = x - q * m                                      # exact: integers below 2^53
    r = np.where(r < 0, r + m, np.where(r >= m, r - m, r))
    return np.where(r > 127, r - m, r).astype(np.int64)


def normalise(v):
    for j in range(3):
        c = np.floor(v[j] / TWO32)
        v[j] = v[j] - c * TWO32
        v[j + 1] = v[j + 1] + c
    return v


def limbs(v):
    return [float((v >> (32 * j)) & 0xFFFFFFFF) for j in range(4)]


def emulate(X, Y):
    """(FP64 result, X' Y' rebuilt, X' Y' exact as Python ints, exponents)."""
    n = X.shape[0]
    N = count(max(256, n))
    ex, Xi = scale(X, axis=1)
    fy, Yi = scale(Y, axis=0)
    Mods = MODULI[:N]
    M = math.prod(Mods)
    mm = limbs(M)
    L = [np.zeros(X.shape) for _ in range(4)]
    worst = 0
    for m in Mods:
        Rx, Ry = residue8(Xi, m), residue8(Yi, m)
        assert Rx.min() >= -128 and Rx.max() <= 127 and Ry.min() >= -128 and Ry.max() <= 127
        P = Rx @ Ry                                          # int64 here; must fit int32
        worst = max(worst, int(np.abs(P).max()))
        Ml = M // m
        y = pow(Ml % m, -1, m)
        t = ((P % m) * y) % m
        ml = limbs(Ml)
        for j in range(4):
            L[j] = L[j] + t.astype(np.float64) * ml[j]
    L = normalise(L)
    sd = ((L[3] * TWO32 + L[2]) * TWO32 + L[1]) * TWO32 + L[0]
    q = np.rint(sd * (1.0 / float(M)))
    V = normalise([L[j] - q * mm[j] for j in range(4)])
    neg = V[3] < 0
    W = normalise([np.where(neg, -V[j], V[j]) for j in range(4)])
    mag = ((W[3] * TWO32 + W[2]) * TWO32 + W[1]) * TWO32 + W[0]
    Z = np.where(neg, -mag, mag)
    exactZ = [[sum(int(Xi[i, k]) * int(Yi[k, j]) for k in range(n)) for j in range(n)] for i in range(n)]
    rebuilt = [[(-1 if neg[i, j] else 1) * sum(int(W[h][i, j]) << (32 * h) for h in range(4))
                for j in range(n)] for i in range(n)]
    return np.ldexp(Z, ex + fy - 2 * B), rebuilt, exactZ, ex, fy, worst, N


def inputs(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n)) * np.exp2(rng.integers(-20, 20, (n, 1)))
    Y = rng.standard_normal((n, n)) * np.exp2(rng.integers(-20, 20, (1, n)))
    X[0, :] = 0.0                                       # a zero row
    X[1, 3] = 2.0 ** -60                                # a tiny entry
    Y[:, 2] = -Y[:, 2]                                  # negative products
    return X, Y


def test_moduli_and_counts():
    for a in range(len(MODULI)):
        for b in range(a + 1, len(MODULI)):
            assert math.gcd(MODULI[a], MODULI[b]) == 1
    assert count(256) == 13
    assert all(count(n) == 14 for n in (512, 1024, 4096, 8192, 65536))
    for n in (256, 8192, 65536):
        M = math.prod(MODULI[:count(n)])
        assert 4 * n * 2 ** (2 * B) < M                 # |X'Y'| <= n 2^2B < M / 4
        assert n * 128 * 128 < 2 ** 31                  # int32 sums of n residue products


@pytest.mark.parametrize("n,seed", [(24, 1), (40, 2)])
def test_limb_reconstruction_is_exact(n, seed):
    X, Y = inputs(n, seed)
    _, rebuilt, exactZ, _, _, worst, N = emulate(X, Y)
    assert worst < 2 ** 31 and N == 13
    assert rebuilt == exactZ


def test_error_bound_against_exact_product():
    n = 32
    X, Y = inputs(n, 3)
    got, _, _, ex, fy, _, _ = emulate(X, Y)
    Xf = [[Fraction(float(v)) for v in row] for row in X]
    Yf = [[Fraction(float(v)) for v in row] for row in Y]
    for i in range(n):
        for j in range(n):
            ref = sum(Xf[i][k] * Yf[k][j] for k in range(n))
            bound = Fraction(n) * Fraction(2) ** int(ex[i, 0] + fy[0, j] - B) + abs(ref) * Fraction(2) ** -50
            assert abs(Fraction(float(got[i, j])) - ref) <= bound, (i, j)


def test_a_planted_off_by_one_modulus_inverse_breaks_it():
    """The reconstruction must depend on every constant: using M_l^-1 + 1 for
    one modulus changes the rebuilt integers."""
    n = 16
    X, Y = inputs(n, 4)
    ex, Xi = scale(X, axis=1)
    fy, Yi = scale(Y, axis=0)
    Mods = MODULI[:13]
    M = math.prod(Mods)
    S = np.zeros((n, n), dtype=object)
    for idx, m in enumerate(Mods):
        P = residue8(Xi, m) @ residue8(Yi, m)
        Ml = M // m
        y = pow(Ml % m, -1, m) + (1 if idx == 5 else 0)
        S = S + ((P % m) * y % m).astype(object) * Ml
    Z = [[int(S[i, j]) - M * round(Fraction(int(S[i, j]), M)) for j in range(n)] for i in range(n)]
    exactZ = [[sum(int(Xi[i, k]) * int(Yi[k, j]) for k in range(n)) for j in range(n)] for i in range(n)]
    assert Z != exactZ
