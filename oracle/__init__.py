"""CPU oracle for truncated Neumann series by radix kernels.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link this package: only the tests, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP library; the only module the
two sides have in common is the seeded input generator package ``workloads``,
which holds none of the method's arithmetic.

Contents
--------
poly        exact rational polynomial algebra: the radix kernels as scalar
            polynomials, the error map and its compositions (Sec. 2.2, Thm 3.1,
            Sec. 4 eq. (4)-(5), Defs 5.1-5.2, Lemmas 5.3-5.5, App. A/B).
coeffs15    the radix-15 coefficient tables: the three-decimal values printed
            in App. B and the polished full-precision table (see polish15).
polish15    regenerates the polished radix-15 table from the printed values by
            minimum-norm Gauss-Newton in mpmath (script; writes
            ``radix15_polished.txt``).
series      the matrix schedules in float64 (or exact Fractions): naive
            Horner, binary splitting, radix-9 telescoping, the general
            radix-kernel (residual) iteration with the radix-15, radix-9,
            quinary and Hensel kernels, quinary and ternary telescoping,
            closed forms, product counts and the residual metric (Sec. 2-6).

Every function cites the passage of the paper it follows.  Parity of the GPU
path is judged against these functions; the functions themselves are pinned
by tests against closed forms, exact rational brute force and the values the
paper prints (``tests/test_oracle_*.py``).
"""

__all__ = ["poly", "coeffs15", "polish15", "series"]
