"""Pins of the oracle's matrix schedules (host only).

References used here are independent of the schedules: explicit powers in
exact rational arithmetic, closed forms, diagonal and nilpotent special cases,
a Jordan block, the paper's printed product counts and residual magnitudes.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

from conftest import golden_rows
from oracle import coeffs15, poly, series
import workloads

EXACT_METHODS = ["binary", "ternary", "quinary", "radix9", "radix9_resid", "quinary_resid", "hensel"]


def _frac_matrix(vals, n):
    M = np.empty((n, n), dtype=object)
    for i, v in enumerate(vals):
        M.flat[i] = Fraction(v)
    return M


@pytest.fixture(scope="module")
def rational3():
    """A nonsymmetric 3 x 3 rational matrix with spectral radius < 1."""
    return _frac_matrix(["1/3", "-1/5", "0", "1/7", "1/4", "1/9", "0", "-1/6", "1/2"], 3)


# --- counts ---------------------------------------------------------------

def test_counts_reproduce_table2():
    cols = {"binary": 1, "quinary": 2, "radix9": 3, "radix15": 4}
    for row in golden_rows("table2_counts.txt"):
        k = int(row[0])
        for method, c in cols.items():
            if row[c] != "-":
                assert series.plan(k, method)[2] == int(row[c]), (k, method)


def test_count_example_and_coefficients():
    rows = golden_rows("count_examples.txt")
    k, r9, b = (int(x) for x in rows[0])
    assert series.plan(k, "radix9")[2] == r9
    assert series.lei_nakamura_count(k) == b
    for row in rows[1:]:
        _, method, coef = row
        per_level = series.PER_LEVEL[method]
        m = series.RADIX[method]
        assert round(per_level / math.log2(m), 2) == float(coef)


@pytest.mark.parametrize("method", list(series.SCHEDULES))
def test_products_performed_equal_formula(method):
    A = workloads.symmetric(8, 0.5, 0).A
    for k in (1, 2, 9, 10, 81, 82):
        _, rep = series.evaluate(A, k, method)
        k_eff, t, g = series.plan(k, method)
        assert rep["products"] == g and rep["k_eff"] == k_eff and rep["levels"] == t


def test_kernel_product_counts_meet_lower_bound():
    """mu_m >= ceil(log2(m - 1)) (Sec. 2.2), met with equality by the kernels."""
    B = workloads.symmetric(6, 0.5, 0).A
    for kern, m in ((series.kernel_quinary, 5), (series.kernel_radix9, 9),
                    (lambda X, mm: series.kernel_radix15(X, mm, coeffs15.polished()), 15)):
        mm = series._Counter()
        kern(B, mm)
        assert mm.n == math.ceil(math.log2(m - 1))


# --- exact rational brute force --------------------------------------------

@pytest.mark.parametrize("method", EXACT_METHODS + ["naive"])
def test_exact_methods_equal_brute_force_bit_for_bit(method, rational3):
    for k in (1, 5, 9, 27, 81):
        S, rep = series.evaluate(rational3, k, method)
        ref = series.brute_force(rational3, rep["k_eff"])
        assert all(S.flat[i] == ref.flat[i] for i in range(9)), (method, k)


def test_naive_powers_equals_horner(rational3):
    a, _ = series.naive_horner(rational3, 20)
    b, _ = series.naive_powers(rational3, 20)
    assert all(a.flat[i] == b.flat[i] for i in range(9))


def test_planted_wrong_kernel_is_caught(rational3):
    """A radix-9 schedule with one wrong post-add coefficient fails the pin."""
    def bad_kernel(B, mm):
        T = series.kernel_radix9(B, mm)
        U = B @ B
        return T + Fraction(1, 800) * U
    S, rep = series.telescoping(rational3, 81, "radix9", bad_kernel)
    ref = series.brute_force(rational3, rep["k_eff"])
    assert any(S.flat[i] != ref.flat[i] for i in range(9))


def test_planted_transposed_operand_is_caught(rational3):
    """Using B^T inside the kernel (a transposed operand) breaks equality."""
    def transposed(B, mm):
        return series.kernel_radix9(B.T.copy(), mm)
    S, rep = series.telescoping(rational3, 81, "radix9", transposed)
    ref = series.brute_force(rational3, rep["k_eff"])
    assert any(S.flat[i] != ref.flat[i] for i in range(9))


def test_general_iteration_residual_is_error_map_iterate():
    """Lemma 5.9 (1): R_n = E^[n](A), in exact arithmetic, for the radix-15
    kernel (rounded doubles taken as exact rationals), n = 1, 2.  The right
    side is the polynomial E^[n] from the kernel algebra evaluated at A."""
    A = _frac_matrix(["1/4", "-1/3", "1/5", "1/6"], 2)
    c28 = coeffs15.polished()
    f = poly.radix15_poly(c28)
    I = series._eye(A)
    for n in (1, 2):
        Y, rep = series.general_radix(A, 15 ** n, "radix15",
                                      lambda B, mm: series.kernel_radix15(B, mm, c28))
        R = I - (I - A) @ Y
        En = poly.iterate_error_map(f, n)
        X = np.empty_like(A)          # Horner evaluation of E^[n] at A
        X[:, :] = Fraction(0)
        for c in reversed(En):
            X = X @ A + c * I
        assert all(R.flat[i] == X.flat[i] for i in range(4)), n


def test_exact_kernel_in_framework_equals_telescoping(rational3):
    """Sec. 5.5: with f = T_m, R_n = A^(m^n) and the framework reproduces the
    telescoping result exactly."""
    a, _ = series.radix9(rational3, 81)
    b, _ = series.radix9_resid(rational3, 81)
    assert all(a.flat[i] == b.flat[i] for i in range(9))


def test_hensel_equals_binary(rational3):
    """Sec. 5.5: Hensel lifting (f = 1 + z) gives binary splitting's S_{2^t}."""
    a, _ = series.hensel(rational3, 64)
    b, _ = series.binary(rational3, 64)
    assert all(a.flat[i] == b.flat[i] for i in range(9))


# --- float64 against closed forms ---------------------------------------------

@pytest.fixture(scope="module")
def sym64():
    return workloads.symmetric(64, 0.9, 11)


@pytest.mark.parametrize("method", EXACT_METHODS + ["naive"])
def test_fp64_matches_spectral_closed_form(method, sym64):
    S, rep = series.evaluate(sym64.A, 81, method)
    ref = series.spectral_form(sym64.Q, sym64.lam, rep["k_eff"])
    assert series.rel_fro(S, ref) < 1e-13


def test_fp64_closed_form_agrees_with_spectral(sym64):
    a = series.closed_form(sym64.A, 200)
    b = series.spectral_form(sym64.Q, sym64.lam, 200)
    assert series.rel_fro(a, b) < 1e-13


def test_spectral_columns_subset(sym64):
    cols = np.array([0, 5, 63])
    full = series.spectral_form(sym64.Q, sym64.lam, 81)
    part = series.spectral_form(sym64.Q, sym64.lam, 81, cols=cols)
    assert np.allclose(full[:, cols], part, rtol=0, atol=1e-13)


@pytest.mark.parametrize("method", EXACT_METHODS + ["radix15"])
def test_diagonal_reduces_to_scalar_geometric_series(method):
    lam = np.array([0.9, -0.8, 0.5, 0.0, -0.3, 0.75])
    # radix-15 is an iteration whose result equals S_k only once E^[t](lam)
    # is below rounding (Lemma 5.9); three levels are enough for |lam| <= 0.9
    k = 3375 if method == "radix15" else 81
    S, rep = series.evaluate(np.diag(lam), k, method)
    k = rep["k_eff"]
    for i, x in enumerate(lam):
        s = 0.0
        for j in range(k):          # the scalar sum written out
            s += x ** j
        assert abs(S[i, i] - s) < 1e-12 * abs(s) + 1e-14
    assert np.count_nonzero(S - np.diag(np.diag(S))) == 0


@pytest.mark.parametrize("method", EXACT_METHODS + ["naive", "radix15"])
def test_nilpotent_gives_exact_inverse(method):
    """Strictly upper triangular A: A^n = 0, so S_k = (I - A)^{-1} for k >= n."""
    rng = np.random.default_rng(3)
    n = 7
    A = np.triu(rng.uniform(-1, 1, (n, n)), 1)
    S, _ = series.evaluate(A, 81, method)
    inv = np.linalg.inv(np.eye(n) - A)
    assert series.rel_fro(S, inv) < 1e-13


def _jordan_sum(lam, n, k):
    """S_k(lam I + N) for the n x n shift N: entry (i, i+j) is
    sum_{r<k} C(r, j) lam^(r-j)  (derivative of the geometric sum / j!)."""
    S = np.zeros((n, n))
    for j in range(n):
        v = sum(math.comb(r, j) * lam ** (r - j) for r in range(j, k))
        for i in range(n - j):
            S[i, i + j] = v
    return S


@pytest.mark.parametrize("method", EXACT_METHODS + ["naive"])
def test_jordan_block_nonnormal(method):
    """Nonnormal test (stands in for Sec. 6's upper triangular matrices)."""
    n, lam = 6, 0.7
    A = lam * np.eye(n) + np.eye(n, k=1)
    S, rep = series.evaluate(A, 81, method)
    ref = _jordan_sum(lam, n, rep["k_eff"])
    assert series.rel_fro(S, ref) < 1e-12


def test_radix15_converges_inside_its_basin(sym64):
    S, rep = series.radix15(sym64.A, 3375)
    ref = series.spectral_form(sym64.Q, sym64.lam, 4096)   # S_inf to fp64 here
    assert series.rel_fro(S, ref) < 1e-13
    assert series.residual_fro(sym64.A, S) < 1e-12
    assert rep["level_norms"][-1] < 1e-12


def test_radix15_printed_table_floors():
    """The three-decimal table stalls: its prefix error 2.8e-3 leaves a
    residual floor many orders above fp64 (the polished table does not)."""
    w = workloads.symmetric(64, 0.9, 12)
    S, _ = series.radix15(w.A, 3375, c28=coeffs15.PRINTED)
    assert series.residual_fro(w.A, S) > 1e-4
    S2, _ = series.radix15(w.A, 3375)
    assert series.residual_fro(w.A, S2) < 1e-12


@pytest.mark.slow
def test_residual_magnitudes_match_table4_in_distribution():
    """Table 4 (d = 500, rho = 0.9): the exact methods' residuals are
    ||A^k||_F of the paper's random matrix, so compare orders of magnitude."""
    w = workloads.symmetric(500, 0.9, 21)
    for method, k, printed in golden_rows("table4_residuals.txt"):
        S, rep = series.evaluate(w.A, int(k), method)
        assert rep["k_eff"] == int(k)
        r = series.residual_fro(w.A, S)
        printed = float(printed)
        if printed > 1e-10:
            assert printed / 5 < r < printed * 5, (method, k, r)
        else:
            assert r < 1e-12, (method, k, r)


# --- exact S_k for any k (mixed radix with additive steps) ---------------------

def test_mixed_equals_brute_force_for_every_k_bit_for_bit(rational3):
    """mixed gives S_k itself, not S_k_eff: every k from 1 to 60 and a few
    beyond, in exact rational arithmetic against explicit powers.  A wrong
    index in the additive step (S_n + A^(n+1)) or a dropped final step fails."""
    P = rational3.copy()
    powers = [series._eye(rational3)]
    for _ in range(130):
        powers.append(powers[-1] @ rational3)
    prefix = [powers[0]]
    for j in range(1, 130):
        prefix.append(prefix[-1] + powers[j])
    for k in list(range(1, 61)) + [81, 82, 100, 127, 128]:
        S, rep = series.mixed(P, k)
        assert (S == prefix[k - 1]).all(), k
        assert rep["k_eff"] == k


def _dijkstra_costs(K):
    """Independent optimum: shortest paths over n = 1..K with edges n -> m n
    (cost mu_m + 2 for the exact kernels) and n -> n + 1 (cost 1); the final
    additive step is free after at least one product."""
    import heapq
    cost = {2: 2, 3: 3, 5: 4, 9: 5}
    dist = [math.inf] * (K + 1)
    dist[1] = 0
    heap = [(0, 1)]
    while heap:
        d, n = heapq.heappop(heap)
        if d > dist[n]:
            continue
        edges = [(n + 1, 1)] + [(n * m, c) for m, c in cost.items()]
        for v, c in edges:
            if v <= K and d + c < dist[v]:
                dist[v] = d + c
                heapq.heappush(heap, (d + c, v))
    final = {1: 0}
    for k in range(2, K + 1):
        free_last = dist[k - 1] if k - 1 >= 2 else dist[k - 1] + 1
        final[k] = min(dist[k], free_last)
    return final


def test_mixed_plan_is_optimal_against_shortest_paths():
    K = 3000
    ref = _dijkstra_costs(K)
    for k in range(1, K + 1):
        products, steps = series.mixed_plan(k)
        assert products == ref[k], k
        # the plan reaches k: replay it
        n = 1
        for s in steps:
            n = n + 1 if s == 1 else n * s
        assert n == k


def test_mixed_never_costs_more_than_the_pure_radices_at_their_own_k():
    for m, method in ((2, "binary"), (3, "ternary"), (5, "quinary"), (9, "radix9")):
        for t in range(1, 8):
            k = m ** t
            assert series.mixed_plan(k)[0] <= series.plan(k, method)[2], (method, k)
    # k = 3375 = 15^3: exact S_3375 in fewer products than radix-9 (k_eff 6561)
    assert series.mixed_plan(3375)[0] < series.plan(3375, "radix9")[2]


def test_mixed_closed_form_large_k():
    w = workloads.symmetric(40, 0.97, 11)
    for k in (1000, 3375, 4097, 12345):
        S, rep = series.mixed(w.A, k)
        ref = series.closed_form(w.A, k)
        assert series.rel_fro(S, ref) < 1e-12, k
        assert rep["products"] == series.mixed_plan(k)[0]


def test_radix15c_converges_where_radix15_diverges():
    """Nonsymmetric N(0,1)/sqrt(n) scaled to rho_hat = 0.99: the App. B kernel's
    residual iteration grows (|E(-0.99)| > 0.99), the contraction-aware kernel
    reaches the closed form (I - A)^{-1} (I - A^k) at k = 15^3."""
    g = workloads.gaussian(96, 0.99, 17)
    ref = series.closed_form(g.A, 3375)
    S_c, rep_c = series.radix15c(g.A, 3375)
    S_b, rep_b = series.radix15(g.A, 3375)
    assert series.rel_fro(S_c, ref) < 1e-12
    assert rep_c["level_norms"][-1] < 1e-10
    assert rep_b["level_norms"][-1] > rep_b["level_norms"][0] > 1.0
    assert rep_c["products"] == rep_b["products"] == 18
