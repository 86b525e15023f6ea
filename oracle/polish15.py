"""Regenerate the polished radix-15 coefficient table (test infrastructure).

Usage:  python -m oracle.polish15 [--check]

Starting point: the 28 coefficients printed in App. B (three decimals).
Target: the 15 prefix conditions of Sec. 4.2, [T15~]_j = 1 for j = 0..14,
where T15~ is the circuit of Sec. 4.1, eq. (4)-(5).

Method: minimum-norm Gauss-Newton in mpmath at 60 significant digits,
    x <- x - J^T (J J^T)^{-1} r(x),    r_j(x) = [T15~(x)]_j - 1,
with the 15 x 28 Jacobian J computed exactly by forward-mode differentiation
of the circuit (product rule on every P_i = L_i R_i).  With 28 unknowns and
15 equations the solution set is a manifold; the minimum-norm step moves the
printed point onto it without leaving the rounding box of the printed digits.

The result is rounded to the nearest doubles and written to
``radix15_polished.txt`` together with the exact-rational prefix error of the
rounded doubles and the spillover coefficients a15, a16 (Sec. 4.2).
``--check`` recomputes the table and fails if it differs from the file.
"""

import argparse
import sys

import mpmath as mp

from . import coeffs15, poly

mp.mp.dps = 60
N_EQ = 15          # prefix conditions j = 0..14
N_PAR = 28


def _circuit_with_jacobian(x):
    """Coefficients of T15~(z) and of d T15~ / d x_p for every parameter p.

    Each basis polynomial is carried as (value, [d value / d x_p]).
    Polynomials are lists of mpf, index = degree.
    """
    def padd(a, b):
        n = max(len(a), len(b))
        return [(a[i] if i < len(a) else 0) + (b[i] if i < len(b) else 0) for i in range(n)]

    def pscale(c, a):
        return [c * v for v in a]

    def pmul(a, b):
        if not a or not b:
            return []
        out = [mp.mpf(0)] * (len(a) + len(b) - 1)
        for i, u in enumerate(a):
            for j, v in enumerate(b):
                out[i + j] += u * v
        return out

    zero = lambda: [[] for _ in range(N_PAR)]  # noqa: E731
    one = ([mp.mpf(1)], zero())
    B = ([mp.mpf(0), mp.mpf(1)], zero())
    P1 = ([mp.mpf(0), mp.mpf(0), mp.mpf(1)], zero())   # P1 = B^2
    basis = [one, B, P1]

    def lincomb(offset, width):
        val, der = [], zero()
        for w in range(width):
            c = x[offset + w]
            bv, bd = basis[w]
            val = padd(val, pscale(c, bv))
            der[offset + w] = padd(der[offset + w], bv)      # d/d c
            for p in range(N_PAR):
                if bd[p]:
                    der[p] = padd(der[p], pscale(c, bd[p]))
        return val, der

    pos = 0
    for width in (3, 4, 5):
        Lv, Ld = lincomb(pos, width)
        Rv, Rd = lincomb(pos + width, width)
        pos += 2 * width
        Pv = pmul(Lv, Rv)
        Pd = [padd(pmul(Ld[p], Rv), pmul(Lv, Rd[p])) for p in range(N_PAR)]
        basis.append((Pv, Pd))

    # T15~ = I + g1 B + g2 P1 + g3 P2 + g4 P3 + P4
    val, der = list(one[0]), zero()
    for gi, bidx in zip(range(24, 28), (1, 2, 3, 4)):
        g = x[gi]
        bv, bd = basis[bidx]
        val = padd(val, pscale(g, bv))
        der[gi] = padd(der[gi], bv)
        for p in range(N_PAR):
            if bd[p]:
                der[p] = padd(der[p], pscale(g, bd[p]))
    P4v, P4d = basis[5]
    val = padd(val, P4v)
    for p in range(N_PAR):
        der[p] = padd(der[p], P4d[p])
    return val, der


def residual_and_jacobian(x):
    val, der = _circuit_with_jacobian(x)
    r = mp.matrix(N_EQ, 1)
    J = mp.matrix(N_EQ, N_PAR)
    for j in range(N_EQ):
        r[j] = (val[j] if j < len(val) else 0) - 1
        for p in range(N_PAR):
            J[j, p] = der[p][j] if j < len(der[p]) else 0
    return r, J


def polish(x0, iters: int = 12, tol=mp.mpf("1e-55")):
    """Minimum-norm Gauss-Newton from x0; returns (x, history of max|r|)."""
    x = [mp.mpf(v) for v in x0]
    hist = []
    for _ in range(iters):
        r, J = residual_and_jacobian(x)
        rmax = max(abs(r[j]) for j in range(N_EQ))
        hist.append(rmax)
        if rmax < tol:
            break
        JJt = J * J.T
        y = mp.lu_solve(JJt, r)
        dx = J.T * y
        x = [x[p] - dx[p] for p in range(N_PAR)]
    return x, hist


def build_table():
    x, hist = polish(coeffs15.PRINTED)
    doubles = [float(v) for v in x]          # round to nearest double
    f = poly.radix15_poly(doubles)           # exact rational composition
    return doubles, hist, f


def render(doubles, hist, f) -> str:
    pe = poly.prefix_error(f, 15)
    lines = [
        "# Polished radix-15 coefficients (circuit of Sec. 4.1, eq. (4)-(5)).",
        "# Written by `python -m oracle.polish15` from the App. B values by",
        "# minimum-norm Gauss-Newton on the prefix conditions of Sec. 4.2.",
        f"# Gauss-Newton max|r| per iteration: {' '.join(mp.nstr(h, 3) for h in hist)}",
        f"# exact prefix error of these doubles, max_j<=14 |[f]_j - 1| = {float(pe):.3e}",
        f"# spillover a15 = {float(poly.coeff(f, 15)):.12f}  a16 = {float(poly.coeff(f, 16)):.12f}"
        f"  degree = {len(f) - 1}",
        f"# c = 1 - a15 = {float(1 - poly.coeff(f, 15)):.12f}",
        "# name  hex-double  decimal  printed",
    ]
    for name, v, pr in zip(coeffs15.NAMES, doubles, coeffs15.PRINTED):
        lines.append(f"{name:8s} {v.hex():24s} {v!r:24s} {pr}")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--check", action="store_true")
    args = ap.parse_args(argv)
    text = render(*build_table())
    if args.check:
        with open(coeffs15.POLISHED_PATH) as fh:
            ok = fh.read() == text
        print("radix15_polished.txt is", "up to date" if ok else "STALE")
        return 0 if ok else 1
    with open(coeffs15.POLISHED_PATH, "w") as fh:
        fh.write(text)
    sys.stdout.write(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
