"""Truncated Neumann series schedules, written plainly (test infrastructure).

Every function takes a square matrix A with rho(A) < 1 and a series length k
and returns an approximation of S_k(A) = I + A + ... + A^(k-1) (eq. (1)),
together with a small report.  The arithmetic is float64 NumPy; the same code
runs on ``dtype=object`` arrays of ``fractions.Fraction`` so that tiny cases
can be checked bit for bit against brute force.  Products go through
``numpy.matmul`` (one library primitive per matrix product); there is no
blocking, fusion or reordering beyond what the paper's steps state.

Schedules round k up to the smallest pure power of the radix, k_eff >= k,
because the paper evaluates only k = m^t (Sec. 6, setup); the report carries
k_eff.  The exception is ``mixed``, which evaluates S_k for any k exactly by
combining radix updates with the additive split of the series.  Product counts follow the literal schedules, including the product
with S_1 = I and the last power or residual update, which is how the paper's
Table 2 counts them.
"""

from fractions import Fraction
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import coeffs15

# ---------------------------------------------------------------------------
# helpers that work for float64 and for Fraction (object) matrices
# ---------------------------------------------------------------------------


def _exact(A: np.ndarray) -> bool:
    return A.dtype == object


def _eye(A: np.ndarray) -> np.ndarray:
    n = A.shape[0]
    if _exact(A):
        I = np.empty((n, n), dtype=object)
        I[:, :] = Fraction(0)
        for i in range(n):
            I[i, i] = Fraction(1)
        return I
    return np.eye(n, dtype=A.dtype)


def _c(x, A: np.ndarray):
    """A scalar coefficient in the arithmetic of A (exact value for Fractions)."""
    if _exact(A):
        return x if isinstance(x, Fraction) else Fraction(x)
    return float(x)


def _fro(X: np.ndarray) -> float:
    if _exact(X):
        return float(sum(v * v for v in X.flat)) ** 0.5
    return float(np.linalg.norm(X, "fro"))


class _Counter:
    """Counts matrix products; each call is one n x n x n GEMM."""

    def __init__(self):
        self.n = 0

    def __call__(self, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
        self.n += 1
        return X @ Y


def _levels(k: int, m: int) -> int:
    """Smallest t with m^t >= k (integer arithmetic, no logarithms)."""
    if k < 1:
        raise ValueError("k must be >= 1")
    t, p = 0, 1
    while p < k:
        p *= m
        t += 1
    return t


# ---------------------------------------------------------------------------
# product counts (Sec. 2.1-2.2 cost model; Sec. 5.4 eq. (9); Table 2)
# ---------------------------------------------------------------------------

RADIX = {"binary": 2, "ternary": 3, "quinary": 5, "radix9": 9, "radix15": 15, "radix15c": 15,
         "radix9_resid": 9, "quinary_resid": 5, "hensel": 2}
# products per update: mu_m + 2 (kernel + concatenation + power/residual)
PER_LEVEL = {"binary": 2, "ternary": 3, "quinary": 4, "radix9": 5, "radix15": 6, "radix15c": 6,
             "radix9_resid": 5, "quinary_resid": 4, "hensel": 2}


def plan(k: int, method: str) -> Tuple[int, int, int]:
    """(k_eff, levels, products) of the literal schedule.

    naive: k - 1 products (Sec. 2.1).  Radix-m methods: t = ceil(log_m k)
    levels of mu_m + 2 products each (Sec. 2.2 cost model, Sec. 5.4).
    mixed: k exactly; levels counts its radix updates.
    """
    if k < 1:
        raise ValueError("k must be >= 1")
    if method == "naive":
        return k, k - 1, k - 1
    if method == "mixed":
        products, steps = mixed_plan(k)
        return k, sum(1 for s in steps if s > 1), products
    m = RADIX[method]
    t = _levels(k, m)
    return m ** t, t, PER_LEVEL[method] * t


# ---------------------------------------------------------------------------
# exact S_k for any k: radix updates and the additive step
# ---------------------------------------------------------------------------
# A radix-m update (S_n, A^n) -> (S_mn, A^mn) costs mu_m + 2 products with an
# exact kernel: binary (mu_2 = 0, T_2 = I + B), ternary (mu_3 = 1), quinary
# (mu_5 = 2, Sec. 2.3) and radix-9 (mu_9 = 3, Thm 3.1).  The additive step
# (S_n, A^n) -> (S_{n+1}, A^{n+1}) takes the series split at n,
# S_{n+r} = S_n + A^n S_r, with r = 1 (S_1 = I), so S_{n+1} = S_n + A^n, and
# A^{n+1} = A A^n: one product.  When the additive step is the last step and
# a product came before it, it needs no new power and costs nothing (the sum
# rides on the previous product).  With nothing before it (k = 2) it is
# counted as one product.

MIXED_COST = {9: 5, 5: 4, 3: 3, 2: 2}


def _mixed_best(n: int, memo: Dict[int, Tuple[int, int]]) -> Tuple[int, int]:
    """(products, choice) to reach (S_n, A^n) from (S_1, A^1) = (I, A).
    choice 0: n - 1 additive steps from 1; choice m: reach n // m, one
    radix-m update, then n % m additive steps.  (Additive steps after a
    radix-m update are fewer than m in an optimal plan: m of them cost more
    than one additive step before the update.)  Ties keep the earlier
    option, in the order: additive chain, m = 9, 5, 3, 2."""
    if n in memo:
        return memo[n]
    best = (n - 1, 0)
    for m in (9, 5, 3, 2):
        if n >= m:
            c = _mixed_best(n // m, memo)[0] + MIXED_COST[m] + n % m
            if c < best[0]:
                best = (c, m)
    memo[n] = best
    return best


def _mixed_steps(n: int, memo) -> List[int]:
    choice = _mixed_best(n, memo)[1]
    if choice == 0:
        return [1] * (n - 1)
    return _mixed_steps(n // choice, memo) + [choice] + [1] * (n % choice)


def mixed_plan(k: int) -> Tuple[int, List[int]]:
    """(products, steps) of the cheapest exact plan for S_k; a step is a
    radix m in {2, 3, 5, 9} or 1 for the additive step.  The last additive
    step is free after a product.  Same tie order as _mixed_best, with the
    additive chain from 1 first."""
    if k < 1:
        raise ValueError("k must be >= 1")
    if k == 1:
        return 0, []
    memo: Dict[int, Tuple[int, int]] = {}
    best = (1 if k == 2 else k - 2, 0)
    for m in (9, 5, 3, 2):
        if k >= m:
            r = k % m
            c = _mixed_best(k // m, memo)[0] + MIXED_COST[m] + max(r - 1, 0)
            if c < best[0]:
                best = (c, m)
    m = best[1]
    if m == 0:
        return best[0], [1] * (k - 1)
    return best[0], _mixed_steps(k // m, memo) + [m] + [1] * (k % m)


def lei_nakamura_count(k: int) -> int:
    """2 log2 k - 1 products (Lei-Nakamura row of Table 3), with log2 k
    rounded up; the paper's k = 9^10 example quotes 63 for binary."""
    return 2 * _levels(k, 2) - 1


# ---------------------------------------------------------------------------
# radix kernels as matrix circuits: B -> (T(B), products used)
# ---------------------------------------------------------------------------


def kernel_quinary(B: np.ndarray, mm: _Counter) -> np.ndarray:
    """Gustafsson's mu_5 = 2 circuit (Sec. 2.3; App. A):
    U = B^2, V = U (B + U), T5 = I + B + U + V."""
    U = mm(B, B)
    V = mm(U, B + U)
    return _eye(B) + B + U + V


def kernel_radix9(B: np.ndarray, mm: _Counter) -> np.ndarray:
    """Theorem 3.1: T9(B) in three products."""
    c = lambda x: _c(x, B)  # noqa: E731
    U = mm(B, B)                                             # MM1
    V = mm(U, B + c(2) * U)                                  # MM2
    P = c(Fraction(3, 20)) * B + c(2) * U + V
    Q = c(Fraction(11, 40)) * B - c(Fraction(1, 8)) * U + c(Fraction(1, 4)) * V
    W = mm(P, Q)                                             # MM3
    return W + _eye(B) + B + c(Fraction(767, 800)) * U + c(Fraction(15, 32)) * V


def kernel_radix15(B: np.ndarray, mm: _Counter, c28: Sequence[float]) -> np.ndarray:
    """The four-product circuit of Sec. 4.1, eq. (4)-(5):
    P1 = B^2; P_i = L_i R_i with L_i, R_i linear combinations of
    {I, B, P1, ..., P_{i-1}} (i = 2, 3, 4);
    T15~ = I + g1 B + g2 P1 + g3 P2 + g4 P3 + P4."""
    c = [_c(x, B) for x in c28]
    basis = [_eye(B), B, mm(B, B)]
    pos = 0
    for width in (3, 4, 5):
        L = sum(c[pos + w] * basis[w] for w in range(width))
        R = sum(c[pos + width + w] * basis[w] for w in range(width))
        pos += 2 * width
        basis.append(mm(L, R))
    g = c[24:28]
    return basis[0] + g[0] * basis[1] + g[1] * basis[2] + g[2] * basis[3] + g[3] * basis[4] + basis[5]


def kernel_hensel(B: np.ndarray, mm: _Counter) -> np.ndarray:
    """f(z) = 1 + z, mu_2 = 0 (Sec. 5.5, Hensel lifting)."""
    return _eye(B) + B


# ---------------------------------------------------------------------------
# schedules
# ---------------------------------------------------------------------------


def _report(method, k, k_eff, levels, mm, norms):
    return {"method": method, "k": k, "k_eff": k_eff, "levels": levels,
            "products": mm.n, "level_norms": norms}


def naive_horner(A: np.ndarray, k: int):
    """Naive evaluation in Horner form, k - 1 products (Sec. 2.1):
    S <- I + A S, starting from S = I."""
    mm = _Counter()
    I = _eye(A)
    S = I.copy()
    for _ in range(k - 1):
        S = I + mm(A, S)
    return S, _report("naive", k, k, k - 1, mm, [])


def naive_powers(A: np.ndarray, k: int):
    """Naive evaluation as the paper words it: accumulate I, A, A^2, ...
    (Sec. 2.1).  Used only as a second definition in tests."""
    mm = _Counter()
    S = _eye(A)
    P = _eye(A)
    for j in range(1, k):
        P = A.copy() if j == 1 else mm(P, A)
        S = S + P
    return S, _report("naive_powers", k, k, k - 1, mm, [])


def binary(A: np.ndarray, k: int):
    """Binary splitting (Sec. 2.1; Sec. 6 setup (i)): per level
    A^{2n} = A^n A^n and S_{2n} = S_n (I + A^n); 2 ceil(log2 k) products."""
    k_eff, t, _ = plan(k, "binary")
    mm = _Counter()
    I = _eye(A)
    S, P = I.copy(), A.copy()
    norms = []
    for _ in range(t):
        S_next = mm(S, I + P)
        P = mm(P, P)
        S = S_next
        norms.append(_fro(P))
    return S, _report("binary", k, k_eff, t, mm, norms)


def ternary(A: np.ndarray, k: int):
    """Ternary splitting (Sec. 2.1): A^{2n} = A^n A^n, A^{3n} = A^{2n} A^n,
    S_{3n} = S_n (I + A^n + A^{2n}); 3 log3 k products."""
    k_eff, t, _ = plan(k, "ternary")
    mm = _Counter()
    I = _eye(A)
    S, P = I.copy(), A.copy()
    norms = []
    for _ in range(t):
        P2 = mm(P, P)
        P3 = mm(P2, P)
        S = mm(S, I + P + P2)
        P = P3
        norms.append(_fro(P))
    return S, _report("ternary", k, k_eff, t, mm, norms)


def telescoping(A: np.ndarray, k: int, method: str,
                kernel: Callable[[np.ndarray, _Counter], np.ndarray]):
    """Exact radix-m update (S_n, A^n) -> (S_mn, A^mn) (Sec. 2.2 cost model):
    T = T_m(A^n) by the kernel (mu_m products),
    S_mn = S_n T (block concatenation, eq. (2)),
    A^mn = I - T (I - A^n) = I - T + T A^n (telescoping identity)."""
    k_eff, t, _ = plan(k, method)
    mm = _Counter()
    I = _eye(A)
    S, P = I.copy(), A.copy()
    norms = []
    for _ in range(t):
        T = kernel(P, mm)
        S = mm(S, T)
        P = I - T + mm(T, P)
        norms.append(_fro(P))
    return S, _report(method, k, k_eff, t, mm, norms)


def radix9(A: np.ndarray, k: int):
    """Radix-9 series, 5 log9 k products (Thm 3.1 inside the Sec. 2.2 update)."""
    return telescoping(A, k, "radix9", kernel_radix9)


def quinary(A: np.ndarray, k: int):
    """Quinary series, 4 log5 k products (Sec. 2.3 kernel, Sec. 2.2 update)."""
    return telescoping(A, k, "quinary", kernel_quinary)


def general_radix(A: np.ndarray, k: int, method: str,
                  kernel: Callable[[np.ndarray, _Counter], np.ndarray]):
    """General radix-kernel iteration, eq. (8) (Sec. 5.3):
    M = I - A, Y_0 = I, R_0 = A;
    Y_{n+1} = Y_n f(R_n),  R_{n+1} = I - M Y_{n+1}.
    The residual is recomputed from M (the true residual), not as E(R_n)."""
    k_eff, t, _ = plan(k, method)
    mm = _Counter()
    I = _eye(A)
    M = I - A
    Y, R = I.copy(), A.copy()
    norms = []
    for _ in range(t):
        Fm = kernel(R, mm)
        Y = mm(Y, Fm)
        R = I - mm(M, Y)
        norms.append(_fro(R))
    return Y, _report(method, k, k_eff, t, mm, norms)


def radix15(A: np.ndarray, k: int, c28: Optional[Sequence[float]] = None):
    """Radix-15 in the general framework, 6 log15 k products (Sec. 4 kernel,
    Sec. 5.3 iteration).  Default coefficients: the polished table."""
    c28 = coeffs15.polished() if c28 is None else list(c28)
    return general_radix(A, k, "radix15", lambda B, mm: kernel_radix15(B, mm, c28))


def radix15c(A: np.ndarray, k: int):
    """Radix-15 in the general framework with the contraction-aware table
    (same circuit and schedule as radix15; E(z) = z^15 p(z) with p's
    coefficients nonnegative, so |E(z)| <= |z|^15 on the unit disk)."""
    c28 = coeffs15.contract_polished()
    return general_radix(A, k, "radix15c", lambda B, mm: kernel_radix15(B, mm, c28))


def radix9_resid(A: np.ndarray, k: int):
    """The exact radix-9 kernel run through the general framework (Sec. 5.5,
    exact radix-m special case: then R_n = A^(9^n))."""
    return general_radix(A, k, "radix9_resid", kernel_radix9)


def quinary_resid(A: np.ndarray, k: int):
    return general_radix(A, k, "quinary_resid", kernel_quinary)


def hensel(A: np.ndarray, k: int):
    """Hensel lifting, Y' = Y (I + R) = Y (2I - M Y) (Sec. 5.5, m = 2)."""
    return general_radix(A, k, "hensel", kernel_hensel)


def _kernel_exact(m: int, B: np.ndarray, mm: _Counter) -> np.ndarray:
    """T_m(B) for the exact radices of the mixed schedule."""
    I = _eye(B)
    if m == 2:
        return I + B
    if m == 3:
        return I + B + mm(B, B)
    if m == 5:
        return kernel_quinary(B, mm)
    if m == 9:
        return kernel_radix9(B, mm)
    raise ValueError(f"no exact kernel for radix {m}")


def mixed(A: np.ndarray, k: int):
    """S_k(A) for any k, exactly (no round-up): the steps of mixed_plan from
    (S_1, A^1) = (I, A).  A radix-m step is the Sec. 2.2 update
    (S_mn = S_n T_m(A^n), A^mn = I - T + T A^n); an additive step is
    S_{n+1} = S_n + A^n with A^{n+1} = A A^n, the last one without the power."""
    products, steps = mixed_plan(k)
    mm = _Counter()
    I = _eye(A)
    S, P = I.copy(), A.copy()
    norms = []
    for i, m in enumerate(steps):
        last = i == len(steps) - 1
        if m == 1:
            if last and mm.n > 0:
                S = S + P
            else:
                S, P = S + P, mm(A, P)
        else:
            T = _kernel_exact(m, P, mm)
            S = mm(S, T)
            P = I - T + mm(T, P)
            norms.append(_fro(P))
    assert mm.n == products
    return S, _report("mixed", k, k, len(norms), mm, norms)


SCHEDULES: Dict[str, Callable] = {
    "naive": naive_horner,
    "binary": binary,
    "ternary": ternary,
    "quinary": quinary,
    "radix9": radix9,
    "radix15": radix15,
    "radix15c": radix15c,
    "radix9_resid": radix9_resid,
    "quinary_resid": quinary_resid,
    "hensel": hensel,
    "mixed": mixed,
}


def evaluate(A: np.ndarray, k: int, method: str):
    return SCHEDULES[method](A, k)


# ---------------------------------------------------------------------------
# definitions, closed forms and metrics
# ---------------------------------------------------------------------------


def brute_force(A: np.ndarray, k: int) -> np.ndarray:
    """sum_{j<k} A^j by explicit powers (eq. (1)); for tiny inputs."""
    I = _eye(A)
    S, P = I.copy(), I.copy()
    for _ in range(1, k):
        P = P @ A
        S = S + P
    return S


def closed_form(A: np.ndarray, k: int) -> np.ndarray:
    """(I - A)^{-1} (I - A^k): the geometric-sum identity T_k(A)(I - A) =
    I - A^k (Sec. 2.2) solved for S_k; A^k by numpy's matrix_power."""
    I = np.eye(A.shape[0])
    return np.linalg.solve(I - A, I - np.linalg.matrix_power(A, k))


def spectral_form(Q: np.ndarray, lam: np.ndarray, k: int,
                  cols: Optional[np.ndarray] = None) -> np.ndarray:
    """S_k(Q diag(lam) Q^T) = Q diag((1 - lam^k)/(1 - lam)) Q^T for orthogonal
    Q; ``cols`` selects columns (then the cost is O(n^2) per column)."""
    g = geometric_sum(lam, k)
    QT = Q.T if cols is None else Q.T[:, cols]
    return (Q * g) @ QT


def permutation_form(A: np.ndarray, k: int) -> np.ndarray:
    """sum_{j<k} A^j (eq. (1)) for A with exactly one nonzero per row (e.g. a
    scaled signed permutation), term by term without a matrix product: row i
    of A^j has its one nonzero where row i of A^(j-1) has it, moved along A
    (column col[pos] of row pos) and scaled by that entry.  FP64; exact while
    every sum of terms fits in 53 bits."""
    n = A.shape[0]
    nz = A != 0
    if not np.all(nz.sum(axis=1) == 1):
        raise ValueError("permutation_form needs exactly one nonzero per row")
    col = np.argmax(nz, axis=1)
    val = A[np.arange(n), col]
    S = np.zeros((n, n))
    rows, pos, coef = np.arange(n), np.arange(n), np.ones(n)
    for _ in range(k):
        S[rows, pos] += coef
        coef = coef * val[pos]
        pos = col[pos]
    return S


def geometric_sum(x: np.ndarray, k: int) -> np.ndarray:
    """sum_{j<k} x^j for scalars |x| < 1, as (1 - x^k)/(1 - x)."""
    x = np.asarray(x, dtype=np.float64)
    return (1.0 - x ** k) / (1.0 - x)


def residual_fro(A: np.ndarray, S: np.ndarray) -> float:
    """||I - (I - A) S||_F, the accuracy measure of Sec. 6."""
    I = np.eye(A.shape[0])
    return float(np.linalg.norm(I - (I - A) @ S, "fro"))


def rel_fro(X: np.ndarray, ref: np.ndarray) -> float:
    """Relative Frobenius error ||X - ref||_F / ||ref||_F."""
    return float(np.linalg.norm(np.asarray(X, np.float64) - ref) / np.linalg.norm(ref))


def level_report_names(method: str) -> List[str]:
    """What the per-level norm is: the power A^(m^n) for the exact
    telescoping schedules, the residual R_n for the general iteration."""
    if method in ("radix15", "radix9_resid", "quinary_resid", "hensel"):
        return ["||R_n||_F"]
    return ["||A^(m^n)||_F"]
