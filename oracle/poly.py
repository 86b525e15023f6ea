"""Exact rational polynomial algebra for radix kernels (test infrastructure).

A polynomial is a list of ``fractions.Fraction`` coefficients, index = degree
(``p[j]`` is the coefficient of z**j).  Floats entering this module are turned
into the exact rational value of the double (``Fraction(float)``), so every
result here is exact: no rounding happens anywhere in this file.

The kernels are evaluated with B replaced by the scalar indeterminate z, which
is how the paper states and proves them (a matrix kernel T(B) is the same
polynomial evaluated at B).
"""

from fractions import Fraction
from typing import List, Sequence

Poly = List[Fraction]


def F(x) -> Fraction:
    """Exact rational value of an int, Fraction or double."""
    if isinstance(x, Fraction):
        return x
    if isinstance(x, int):
        return Fraction(x)
    return Fraction(float(x))


def norm(p: Sequence) -> Poly:
    """Drop trailing zero coefficients (the zero polynomial is [])."""
    q = [F(c) for c in p]
    while q and q[-1] == 0:
        q.pop()
    return q


def const(c) -> Poly:
    return norm([F(c)])


def z_pow(j: int) -> Poly:
    return [Fraction(0)] * j + [Fraction(1)]


def add(*ps: Sequence) -> Poly:
    n = max((len(p) for p in ps), default=0)
    out = [Fraction(0)] * n
    for p in ps:
        for j, c in enumerate(p):
            out[j] += F(c)
    return norm(out)


def scale(c, p: Sequence) -> Poly:
    c = F(c)
    return norm([c * F(x) for x in p])


def lincomb(coeffs: Sequence, basis: Sequence[Sequence]) -> Poly:
    """sum_i coeffs[i] * basis[i]."""
    return add(*[scale(c, b) for c, b in zip(coeffs, basis)])


def mul(p: Sequence, q: Sequence) -> Poly:
    if not p or not q:
        return []
    out = [Fraction(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        if a == 0:
            continue
        for j, b in enumerate(q):
            out[i + j] += F(a) * F(b)
    return norm(out)


def compose(f: Sequence, g: Sequence) -> Poly:
    """f(g(z)) by Horner's rule in the polynomial ring."""
    out: Poly = []
    for c in reversed(list(f)):
        out = add(mul(out, g), [F(c)])
    return norm(out)


def truncate(p: Sequence, deg: int) -> Poly:
    """Terms of degree < deg."""
    return norm(list(p)[:deg])


def coeff(p: Sequence, j: int) -> Fraction:
    return F(p[j]) if j < len(p) else Fraction(0)


def evaluate(p: Sequence, x):
    """Horner evaluation at a scalar (Fraction or float)."""
    acc = 0
    for c in reversed(list(p)):
        acc = acc * x + (c if not isinstance(x, float) else float(c))
    return acc


def geometric(m: int) -> Poly:
    """T_m(z) = 1 + z + ... + z^(m-1)  (Sec. 1, the kernel definition)."""
    return [Fraction(1)] * m


# ---------------------------------------------------------------------------
# The kernels as polynomials in z (B -> z)
# ---------------------------------------------------------------------------

def quinary_poly() -> Poly:
    """Gustafsson's radix-5 circuit (Sec. 2.3; App. A, quinary kernel):
    U = B^2, V = U (B + U), T5 = I + B + U + V."""
    B = z_pow(1)
    U = mul(B, B)
    V = mul(U, add(B, U))
    return add(const(1), B, U, V)


# Rational coefficients of Theorem 3.1 (radix-9 kernel in three products).
R9_V_SHIFT = Fraction(2)                       # V = U (B + 2U)
R9_P = (Fraction(3, 20), Fraction(2), Fraction(1))       # P over (B, U, V)
R9_Q = (Fraction(11, 40), Fraction(-1, 8), Fraction(1, 4))  # Q over (B, U, V)
R9_T = (Fraction(1), Fraction(767, 800), Fraction(15, 32))  # T9 adds (B, U, V)


def radix9_poly(p=R9_P, q=R9_Q, t=R9_T, v_shift=R9_V_SHIFT) -> Poly:
    """The radix-9 circuit of Theorem 3.1 evaluated as a polynomial.

    Steps (MM = matrix product):
      U = B^2 (MM1);  V = U (B + 2U) (MM2);
      P = 3/20 B + 2U + V;  Q = 11/40 B - 1/8 U + 1/4 V;  W = P Q (MM3);
      T9 = W + I + B + 767/800 U + 15/32 V.
    The keyword arguments exist so that tests can plant a wrong coefficient
    and see the exactness pin fail.
    """
    B = z_pow(1)
    U = mul(B, B)
    V = mul(U, add(B, scale(v_shift, U)))
    P = lincomb(p, [B, U, V])
    Q = lincomb(q, [B, U, V])
    W = mul(P, Q)
    return add(W, const(1), scale(t[0], B), scale(t[1], U), scale(t[2], V))


def radix15_poly(c28: Sequence) -> Poly:
    """The four-product radix-15 circuit of Sec. 4.1, eq. (4)-(5).

    ``c28`` holds the 28 coefficients in the order
      L2[I,B,P1], R2[I,B,P1], L3[I,B,P1,P2], R3[..], L4[I,B,P1,P2,P3], R4[..],
      gamma1..gamma4,
    i.e. the factors of P_i range over {I, B, P1, ..., P_{i-1}} (reading of the
    basis indexing), and
      T15~ = I + g1 B + g2 P1 + g3 P2 + g4 P3 + P4.
    """
    c = [F(x) for x in c28]
    assert len(c) == 28
    B = z_pow(1)
    basis = [const(1), B, mul(B, B)]            # {I, B, P1}, P1 = B^2
    pos = 0
    for width in (3, 4, 5):                      # factors of P2, P3, P4
        L = lincomb(c[pos:pos + width], basis)
        R = lincomb(c[pos + width:pos + 2 * width], basis)
        pos += 2 * width
        basis.append(mul(L, R))                  # P_i = L_i R_i
    g = c[24:28]
    return add(const(1), scale(g[0], basis[1]), scale(g[1], basis[2]),
               scale(g[2], basis[3]), scale(g[3], basis[4]), basis[5])


def hensel_poly() -> Poly:
    """m = 2 special case of the framework: f(z) = 1 + z (Sec. 5.5)."""
    return [Fraction(1), Fraction(1)]


# ---------------------------------------------------------------------------
# Approximate-kernel theory (Sec. 5.1-5.2)
# ---------------------------------------------------------------------------

def error_map(f: Sequence) -> Poly:
    """E(z) = 1 - (1 - z) f(z)  (Definition 5.2)."""
    return add(const(1), scale(-1, mul([Fraction(1), Fraction(-1)], f)))


def is_approx_kernel(f: Sequence, m: int) -> bool:
    """(1 - z) f(z) = 1 + O(z^m)  (Definition 5.1)."""
    g = mul([Fraction(1), Fraction(-1)], f)
    return all(coeff(g, j) == (1 if j == 0 else 0) for j in range(m))


def prefix_error(f: Sequence, m: int) -> Fraction:
    """max_{0<=j<m} |[f]_j - 1|: how far f is from (1-z)^{-1} mod z^m
    (the quantity bounded in Sec. 4.2)."""
    return max(abs(coeff(f, j) - 1) for j in range(m))


def spillover(f: Sequence, m: int) -> Poly:
    """Terms of f of degree >= m (Definition 5.1), as a list starting at z^m."""
    return [coeff(f, j) for j in range(m, len(f))]


def leading_error_coeff(f: Sequence, m: int) -> Fraction:
    """c = 1 - [f]_m  (Lemma 5.3, error order)."""
    return 1 - coeff(f, m)


def iterate_error_map(f: Sequence, n: int) -> Poly:
    """E^[n](z): n-fold composition, E^[0](z) = z  (Lemma 5.7)."""
    E = error_map(f)
    out = z_pow(1)
    for _ in range(n):
        out = compose(E, out)
    return out


def lift(f: Sequence) -> Poly:
    """One lift of the general radix-kernel summation: f(z) f(E(z))
    (Definition 5.4, eq. (6))."""
    return mul(f, compose(f, error_map(f)))
