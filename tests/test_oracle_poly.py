"""Pins of the oracle's exact kernel algebra (host only).

Each test checks the oracle against something other than itself: the target
polynomial T_m, coefficient vectors and spillover values the paper prints,
identities that hold for any polynomial, or exact rational surrogates.
"""

from fractions import Fraction

import numpy as np
import pytest

from conftest import golden_rows
from oracle import coeffs15, poly, polish15


def _golden_dict(name):
    return {r[0]: r[1:] for r in golden_rows(name)}


# --- radix-9 (Theorem 3.1) -------------------------------------------------

def test_radix9_circuit_equals_T9_exactly():
    assert poly.radix9_poly() == poly.geometric(9)


def test_radix9_intermediate_V():
    """Theorem 3.1 step 2 states V = U (B + 2U) = B^3 + 2 B^4."""
    B = poly.z_pow(1)
    U = poly.mul(B, B)
    V = poly.mul(U, poly.add(B, poly.scale(poly.R9_V_SHIFT, U)))
    assert V == [0, 0, 0, 1, 2]


def test_radix9_factors_match_printed_proof_vectors():
    """The proof lists P, Q as coefficient vectors over B^1..B^4."""
    g = _golden_dict("radix9_proof_vectors.txt")
    B = poly.z_pow(1)
    U = poly.mul(B, B)
    V = poly.add(poly.z_pow(3), poly.scale(2, poly.z_pow(4)))
    P = poly.lincomb(poly.R9_P, [B, U, V])
    Q = poly.lincomb(poly.R9_Q, [B, U, V])
    assert [poly.coeff(P, j) for j in range(1, 5)] == [Fraction(x) for x in g["p"]]
    assert [poly.coeff(Q, j) for j in range(1, 5)] == [Fraction(x) for x in g["q"]]
    # the convolution P Q has coefficient 1 in degrees 5..8 (proof of Thm 3.1)
    W = poly.mul(P, Q)
    assert [poly.coeff(W, j) for j in range(5, 9)] == [1, 1, 1, 1]
    assert poly.R9_T[1] == Fraction(g["t_U"][0]) and float(poly.R9_T[1]) == float(g["t_U"][1])
    assert poly.R9_T[2] == Fraction(g["t_V"][0]) and float(poly.R9_T[2]) == float(g["t_V"][1])


def test_radix9_denominators_divide_800():
    """Remark 3.2: all coefficients are rationals with denominators dividing 800."""
    for c in (*poly.R9_P, *poly.R9_Q, *poly.R9_T):
        assert 800 % Fraction(c).denominator == 0


@pytest.mark.parametrize("which,idx,delta", [
    ("p", 0, Fraction(1, 800)), ("p", 1, Fraction(1, 100)), ("q", 2, Fraction(-1, 64)),
    ("t", 1, Fraction(1, 800)), ("t", 2, Fraction(1, 32)), ("v", 0, Fraction(1, 2)),
])
def test_radix9_planted_mistake_is_caught(which, idx, delta):
    """A wrong coefficient anywhere in the circuit breaks exactness."""
    p, q, t, v = list(poly.R9_P), list(poly.R9_Q), list(poly.R9_T), poly.R9_V_SHIFT
    if which == "p":
        p[idx] += delta
    elif which == "q":
        q[idx] += delta
    elif which == "t":
        t[idx] += delta
    else:
        v += delta
    assert poly.radix9_poly(p, q, t, v) != poly.geometric(9)


def test_radix9_error_map_is_z9():
    """Exact kernels have E(z) = z^m (Lemma 5.3, exact case; Sec. 5.5)."""
    assert poly.error_map(poly.radix9_poly()) == poly.z_pow(9)


# --- quinary and Hensel (Sec. 2.3, Sec. 5.5) --------------------------------

def test_quinary_exact():
    assert poly.quinary_poly() == poly.geometric(5)
    assert poly.error_map(poly.quinary_poly()) == poly.z_pow(5)


def test_hensel_error_map_is_z2():
    assert poly.error_map(poly.hensel_poly()) == poly.z_pow(2)


# --- radix-15 (Sec. 4, App. B) ----------------------------------------------

def _claims():
    return {r[0]: float(r[1]) for r in golden_rows("radix15_claims.txt")}


def test_radix15_printed_table_misses_the_papers_bound():
    """The three-decimal App. B values, composed exactly, give a prefix error
    of 2.8e-3, far above the paper's < 9e-7: the reason the oracle polishes."""
    f = poly.radix15_poly(coeffs15.PRINTED)
    pe = float(poly.prefix_error(f, 15))
    assert 2.5e-3 < pe < 3.2e-3
    assert pe > _claims()["prefix_bound"]


def test_radix15_polished_meets_prefix_bound_and_printed_spillover():
    cl = _claims()
    f = poly.radix15_poly(coeffs15.polished())
    assert float(poly.prefix_error(f, 15)) < 1e-15 < cl["prefix_bound"]
    assert len(f) - 1 == 16                      # degree exactly 16
    assert round(float(poly.coeff(f, 15)), 3) == cl["a15"]
    assert round(float(poly.coeff(f, 16)), 3) == cl["a16"]
    assert round(float(poly.leading_error_coeff(f, 15)), 2) == cl["c"]


def test_radix15_polished_rounds_to_printed_digits():
    """Every polished coefficient lies in the rounding interval of the printed
    three-decimal value (half a unit in the third decimal, plus a hair)."""
    for name, x, p in zip(coeffs15.NAMES, coeffs15.polished(), coeffs15.PRINTED):
        assert abs(x - p) <= 5e-4 + 1e-12, name


def test_polished_table_regenerates():
    doubles, _, _ = polish15.build_table()
    assert doubles == coeffs15.polished()


def test_radix15_is_approximate_kernel():
    """Definition 5.1 with m = 15 holds to the rounding of the doubles; the
    printed table fails it by 3e-3."""
    f = poly.radix15_poly(coeffs15.polished())
    g = poly.mul([Fraction(1), Fraction(-1)], f)
    assert abs(poly.coeff(g, 0) - 1) < 1e-15
    assert all(abs(poly.coeff(g, j)) < 1e-15 for j in range(1, 15))
    assert abs(poly.coeff(g, 15)) > 0.1


# --- contraction-aware radix-15 table ------------------------------------------

def _error_quadratic(c28):
    """(c0, c1, c2) with E(z) = z^15 (c0 + c1 z + c2 z^2) + (prefix rounding), from
    the exact rational composition of the circuit."""
    f = poly.radix15_poly(c28)
    E = poly.error_map(f)
    assert len(E) - 1 == 17
    return f, [poly.coeff(E, 15), poly.coeff(E, 16), poly.coeff(E, 17)]


def test_contract_table_is_prefix_exact_with_nonnegative_error_quadratic():
    """Prefix conditions of Sec. 4.2 to the rounding of the doubles, and
    E(z) = z^15 p(z) with p's coefficients all >= 0.11: |p(z)| <= 1 on the unit
    disk (they sum to 1 exactly up to the prefix rounding)."""
    f, (c0, c1, c2) = _error_quadratic(coeffs15.contract_polished())
    assert float(poly.prefix_error(f, 15)) < 1e-15
    E = poly.error_map(f)
    assert all(abs(poly.coeff(E, j)) < 1e-14 for j in range(15))
    assert min(c0, c1, c2) > Fraction(11, 100)
    assert abs(c0 + c1 + c2 - 1) < 1e-14
    # p's coefficients are 1 - a15, a15 - a16, a16 (Definition 5.2 expanded,
    # exactly so up to the prefix rounding of [f]_14)
    a15, a16 = poly.coeff(f, 15), poly.coeff(f, 16)
    assert abs(c0 - (1 - a15)) < 1e-14 and c1 == a15 - a16 and c2 == a16


def test_contract_table_contracts_where_the_app_b_table_does_not():
    """|E(z)| <= |z|^15 on the unit circle for the new table; the App. B table
    has |E(-0.99)| = 1.32 > 0.99 (the divergence of the rho = 0.99 workload)."""
    _, q = _error_quadratic(coeffs15.contract_polished())
    _, q_b = _error_quadratic(coeffs15.polished())
    th = np.linspace(0, 2 * np.pi, 721)
    z = np.exp(1j * th)
    p = sum(float(c) * z ** i for i, c in enumerate(q))
    assert np.abs(p).max() <= 1 + 1e-12
    r = -0.99
    e_b = abs(r ** 15 * sum(float(c) * r ** i for i, c in enumerate(q_b)))
    e_c = abs(r ** 15 * sum(float(c) * r ** i for i, c in enumerate(q)))
    assert e_b > 1.3 and e_c < 0.99 ** 15


def test_contract_table_regenerates_from_its_start_point():
    """Polishing the stored six-decimal start point reproduces the table, and
    every coefficient is within half a unit of the sixth decimal of it."""
    from oracle import contract15
    assert open(contract15.POLISHED_PATH).read() == contract15.render_polished(coeffs15.contract_start())
    for name, x, s in zip(coeffs15.NAMES, coeffs15.contract_polished(), coeffs15.contract_start()):
        assert abs(x - s) <= 5e-7 + 1e-12, name


@pytest.mark.parametrize("idx", [0, 9, 17, 27])
def test_contract_table_planted_mistake_is_caught(idx):
    c = list(coeffs15.contract_polished())
    c[idx] += 1e-3
    assert float(poly.prefix_error(poly.radix15_poly(c), 15)) > 1e-7


# --- framework lemmas on exact surrogates (Sec. 5.1-5.2) ----------------------

def _surrogate(m=15, a=Fraction(37, 200), b=Fraction(229, 500)):
    """An exact approximate radix-m kernel with rational spillover a z^m + b z^(m+1)."""
    return poly.add(poly.geometric(m), poly.scale(a, poly.z_pow(m)), poly.scale(b, poly.z_pow(m + 1)))


def test_lemma_error_order():
    """Lemma 5.3: E(z) = (1 - a_m) z^m + O(z^{m+1})."""
    a = Fraction(37, 200)
    f = _surrogate(a=a)
    E = poly.error_map(f)
    assert all(poly.coeff(E, j) == 0 for j in range(15))
    assert poly.coeff(E, 15) == 1 - a


@pytest.mark.parametrize("f", [
    poly.radix9_poly(), poly.quinary_poly(), _surrogate(), _surrogate(5, Fraction(1, 3), Fraction(-2, 7)),
    [Fraction(1), Fraction(1, 2), Fraction(-3, 5)],        # not a kernel at all
])
def test_lemma_composition_identity(f):
    """Lemma 5.5: E(E(z)) = 1 - (1 - z) f(z) f(E(z)) for any polynomial f."""
    E = poly.error_map(f)
    lhs = poly.compose(E, E)
    rhs = poly.add(poly.const(1), poly.scale(-1, poly.mul([1, -1], poly.mul(f, poly.compose(f, E)))))
    assert lhs == rhs


def test_lemma_prefix_growth():
    """Lemma 5.6: f(z) f(E(z)) matches (1 - z)^{-1} in its first m^2 coefficients."""
    m = 5
    f = _surrogate(m, Fraction(1, 3), Fraction(-2, 7))
    g = poly.lift(f)
    assert all(poly.coeff(g, j) == 1 for j in range(m * m))
    assert poly.coeff(g, m * m) != 1


@pytest.mark.parametrize("n", [1, 2])
def test_lemma_error_propagation(n):
    """Lemma 5.7: E^[n](z) = c^{(m^n - 1)/(m - 1)} z^{m^n} + O(z^{m^n + 1})."""
    m, a = 5, Fraction(1, 3)
    f = _surrogate(m, a, Fraction(-2, 7))
    c = 1 - a
    En = poly.iterate_error_map(f, n)
    deg = m ** n
    assert all(poly.coeff(En, j) == 0 for j in range(deg))
    assert poly.coeff(En, deg) == c ** ((m ** n - 1) // (m - 1))


def test_polynomial_helpers_against_brute_force_evaluation():
    """compose/mul agree with pointwise evaluation at rational points."""
    f = poly.radix15_poly(coeffs15.polished())
    E = poly.error_map(f)
    for x in (Fraction(1, 3), Fraction(-7, 10), Fraction(9, 10)):
        assert poly.evaluate(E, x) == 1 - (1 - x) * poly.evaluate(f, x)
    g = _surrogate(5, Fraction(1, 3), Fraction(-2, 7))
    Eg = poly.error_map(g)
    for x in (Fraction(1, 3), Fraction(-7, 10)):
        assert poly.evaluate(poly.compose(g, Eg), x) == poly.evaluate(g, poly.evaluate(Eg, x))
        assert poly.evaluate(poly.mul(g, Eg), x) == poly.evaluate(g, x) * poly.evaluate(Eg, x)
