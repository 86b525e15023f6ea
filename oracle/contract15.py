"""Search and polish a contraction-aware radix-15 coefficient table (test infrastructure).

Usage:  python -m oracle.contract15 [--check | --search]

Background.  For a prefix-exact kernel of the Sec. 4.1 circuit, f has degree
16 and [f]_j = 1 for j <= 14 (Sec. 4.2), so the error map of Definition 5.2 is

    E(z) = 1 - (1 - z) f(z) = z^15 p(z),
    p(z) = (1 - a15) + (a15 - a16) z + a16 z^2,      a15 = [f]_15, a16 = [f]_16.

The coefficients of p sum to 1.  When all three are nonnegative,
|p(z)| <= 1 and hence |E(z)| <= |z|^15 on the closed unit disk: the residual
iteration of eq. (8) then contracts every eigenvalue inside the disk as fast
as the exact kernel would.  The App. B kernel has a15 - a16 < 0
(a15 = 0.185, a16 = 0.458): |E(-0.99)| = 0.99^15 |p(-0.99)| = 1.32 > 0.99, so
eigenvalues near -0.99 grow from level to level.

Search.  Among the 28-coefficient circuits satisfying the 15 prefix
conditions, minimise the coefficient norm |x|^2 subject to the margins
a15 - a16 >= 0.12, a16 >= 0.12, 1 - a15 >= 0.12, with SLSQP (scipy) from 40
seeded perturbations (N(0, 0.5^2) per coefficient, seed 2602) of the App. B
point; every result is projected back onto the prefix conditions by
minimum-norm Gauss-Newton in float64, and the feasible result of smallest
norm is kept.  Its coefficients rounded to six decimals are the START table
(``radix15c_start.txt``).

Polish.  START is polished exactly as ``polish15`` polishes App. B (mpmath,
60 digits, minimum-norm Gauss-Newton with the exact Jacobian), and the limit,
rounded to doubles, is ``radix15c_polished.txt``.

--check   re-polishes the stored START and fails if the polished file differs
          (it does not rerun the search).
--search  reruns the search and fails if it does not reproduce START.
With no option both files are (re)written.
"""

import argparse
import os
import sys
from typing import List

import numpy as np

from . import coeffs15, poly, polish15

HERE = os.path.dirname(os.path.abspath(__file__))
START_PATH = os.path.join(HERE, "radix15c_start.txt")
POLISHED_PATH = os.path.join(HERE, "radix15c_polished.txt")
MARGIN = 0.12
SEED = 2602
TRIALS = 40


# --- float64 circuit for the search (the rational one in poly.py is exact but slow)

def _circuit(x: np.ndarray) -> np.ndarray:
    """Coefficients of T15~(z) (degree 16) for the 28 circuit coefficients."""
    basis = [np.array([1.0]), np.array([0.0, 1.0]), np.array([0.0, 0.0, 1.0])]
    pos = 0
    for width in (3, 4, 5):
        L = np.zeros(len(basis[width - 1]))      # degree of the widest basis member
        R = np.zeros_like(L)
        for w in range(width):
            b = basis[w]
            L[:len(b)] += x[pos + w] * b
            R[:len(b)] += x[pos + width + w] * b
        pos += 2 * width
        basis.append(np.convolve(L, R))
    f = np.zeros(17)
    f[0] = 1.0
    for g, b in zip(x[24:28], basis[1:5]):
        f[:len(b)] += g * b
    f[:len(basis[5])] += basis[5]
    return f


def _prefix_residual(x):
    return _circuit(x)[:15] - 1.0


def _spill(x):
    f = _circuit(x)
    return f[15], f[16]


def _project(x: np.ndarray) -> np.ndarray:
    for _ in range(30):
        r = _prefix_residual(x)
        if np.abs(r).max() < 1e-13:
            break
        J = np.empty((15, 28))
        for i in range(28):
            xp = x.copy()
            xp[i] += 1e-7
            J[:, i] = (_prefix_residual(xp) - r) / 1e-7
        x = x - np.linalg.lstsq(J, r, rcond=None)[0]
    return x


def search() -> List[float]:
    import warnings
    from scipy.optimize import minimize
    cons = [{"type": "eq", "fun": _prefix_residual},
            {"type": "ineq", "fun": lambda x: _spill(x)[0] - _spill(x)[1] - MARGIN},
            {"type": "ineq", "fun": lambda x: _spill(x)[1] - MARGIN},
            {"type": "ineq", "fun": lambda x: 1.0 - _spill(x)[0] - MARGIN}]
    x0 = np.array(coeffs15.PRINTED)
    rng = np.random.default_rng(SEED)
    best = None
    for _ in range(TRIALS):
        xs = x0 + rng.normal(0.0, 0.5, 28)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            res = minimize(lambda x: x @ x, xs, method="SLSQP", constraints=cons,
                           bounds=[(-3.0, 3.0)] * 28, options={"maxiter": 500, "ftol": 1e-14})
        x = _project(res.x)
        a15, a16 = _spill(x)
        feasible = (np.abs(_prefix_residual(x)).max() < 1e-12 and a15 - a16 > MARGIN - 1e-6
                    and a16 > MARGIN - 1e-6 and a15 < 1.0 - MARGIN + 1e-6)
        if feasible and (best is None or x @ x < best @ best):
            best = x
    if best is None:
        raise RuntimeError("no feasible kernel found")
    return [round(float(v), 6) for v in best]


# --- files -----------------------------------------------------------------------

def read_table(path: str, column: int) -> List[float]:
    vals = []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                tok = line.split()[column]
                vals.append(float.fromhex(tok) if tok.startswith(("0x", "-0x")) else float(tok))
    if len(vals) != 28:
        raise ValueError(f"{path}: expected 28 coefficients, got {len(vals)}")
    return vals


def render_start(start: List[float]) -> str:
    lines = ["# Contraction-aware radix-15 start point, six decimals (`python -m oracle.contract15`).",
             f"# Seeded SLSQP search (seed {SEED}, {TRIALS} starts): min |x|^2 over the prefix-exact",
             f"# circuits with a15 - a16, a16, 1 - a15 >= {MARGIN}.", "# name  value"]
    lines += [f"{n:8s} {v: .6f}" for n, v in zip(coeffs15.NAMES, start)]
    return "\n".join(lines) + "\n"


def render_polished(start: List[float]):
    x, hist = polish15.polish(start)
    doubles = [float(v) for v in x]
    f = poly.radix15_poly(doubles)               # exact rational composition
    pe = poly.prefix_error(f, 15)
    a15, a16 = poly.coeff(f, 15), poly.coeff(f, 16)
    lines = [
        "# Contraction-aware radix-15 coefficients (circuit of Sec. 4.1, eq. (4)-(5)).",
        "# Written by `python -m oracle.contract15`: the start point polished by minimum-norm",
        "# Gauss-Newton on the prefix conditions of Sec. 4.2.",
        f"# Gauss-Newton max|r| per iteration: {' '.join(polish15.mp.nstr(h, 3) for h in hist)}",
        f"# exact prefix error of these doubles, max_j<=14 |[f]_j - 1| = {float(pe):.3e}",
        f"# spillover a15 = {float(a15):.12f}  a16 = {float(a16):.12f}  degree = {len(f) - 1}",
        f"# E(z) = z^15 (c0 + c1 z + c2 z^2): c0 = {float(1 - a15):.12f}  c1 = {float(a15 - a16):.12f}"
        f"  c2 = {float(a16):.12f}",
        "# name  hex-double  decimal  start",
    ]
    for name, v, s in zip(coeffs15.NAMES, doubles, start):
        lines.append(f"{name:8s} {v.hex():24s} {v!r:24s} {s:.6f}")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    g = ap.add_mutually_exclusive_group()
    g.add_argument("--check", action="store_true")
    g.add_argument("--search", action="store_true")
    args = ap.parse_args(argv)
    if args.check:
        ok = open(POLISHED_PATH).read() == render_polished(read_table(START_PATH, 1))
        print("radix15c_polished.txt is", "up to date" if ok else "STALE")
        return 0 if ok else 1
    start = search()
    if args.search:
        ok = start == read_table(START_PATH, 1)
        print("search", "reproduces" if ok else "does NOT reproduce", "radix15c_start.txt")
        return 0 if ok else 1
    with open(START_PATH, "w") as fh:
        fh.write(render_start(start))
    text = render_polished(start)
    with open(POLISHED_PATH, "w") as fh:
        fh.write(text)
    sys.stdout.write(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
