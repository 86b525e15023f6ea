"""Radix-15 coefficient tables (test infrastructure).

Order of the 28 entries (the circuit of Sec. 4.1, eq. (4)-(5); the factors
of P_i range over {I, B, P1, ..., P_{i-1}}):

    L2[I,B,P1]  R2[I,B,P1]
    L3[I,B,P1,P2]  R3[I,B,P1,P2]
    L4[I,B,P1,P2,P3]  R4[I,B,P1,P2,P3]
    gamma1..gamma4          (T15~ = I + g1 B + g2 P1 + g3 P2 + g4 P3 + P4)

PRINTED is App. B as printed, to three decimals.  Composed exactly, these
rounded values miss the paper's own prefix bound (max_{j<=14} |[f]_j - 1|
< 9e-7, Sec. 4.2) by more than three orders of magnitude, so the kernel the
oracle evaluates is the POLISHED table: the printed point moved by a
minimum-norm Gauss-Newton iteration onto the set of exact prefix solutions
(``polish15.py`` writes it; each entry stays within rounding distance of its
printed value).  The polished table is read from ``radix15_polished.txt``.

A second, contraction-aware table (``contract15.py`` writes it) is another
point of the same prefix-exact set, chosen so that the error map
E(z) = z^15 p(z) has a p with nonnegative coefficients: |E(z)| <= |z|^15 on
the unit disk.  ``contract_start()`` is its six-decimal start point and
``contract_polished()`` the polished doubles.
"""

import os
from typing import List

# App. B, radix-15 explicit circuit (three decimals as printed).
PRINTED: List[float] = [
    0.238, 0.241, 1.574,                 # L2
    0.048, -0.047, 0.889,                # R2
    0.263, 0.919, 0.842, 0.819,          # L3
    0.184, 0.068, 0.134, -1.405,         # R3
    -0.005, -1.385, 0.022, 0.122, 0.275,  # L4
    -0.701, 0.602, -0.624, -0.137, 0.328,  # R4
    0.078, 1.778, 0.664, -0.024,         # gamma1..gamma4
]

NAMES: List[str] = (
    [f"L2_{x}" for x in ("I", "B", "P1")] + [f"R2_{x}" for x in ("I", "B", "P1")]
    + [f"L3_{x}" for x in ("I", "B", "P1", "P2")]
    + [f"R3_{x}" for x in ("I", "B", "P1", "P2")]
    + [f"L4_{x}" for x in ("I", "B", "P1", "P2", "P3")]
    + [f"R4_{x}" for x in ("I", "B", "P1", "P2", "P3")]
    + [f"gamma{i}" for i in range(1, 5)]
)

POLISHED_PATH = os.path.join(os.path.dirname(__file__), "radix15_polished.txt")


CONTRACT_START_PATH = os.path.join(os.path.dirname(__file__), "radix15c_start.txt")
CONTRACT_POLISHED_PATH = os.path.join(os.path.dirname(__file__), "radix15c_polished.txt")


def contract_start() -> List[float]:
    """Six-decimal start point of the contraction-aware table."""
    return _read(CONTRACT_START_PATH, float)


def contract_polished() -> List[float]:
    """The contraction-aware table as doubles."""
    return _read(CONTRACT_POLISHED_PATH, float.fromhex)


def _read(path, conv) -> List[float]:
    vals = []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                vals.append(conv(line.split()[1]))
    if len(vals) != 28:
        raise ValueError(f"{path}: expected 28 coefficients, got {len(vals)}")
    return vals


def polished() -> List[float]:
    """The polished table as doubles (hex-float column of the text file)."""
    vals = []
    with open(POLISHED_PATH) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            name, hexval = line.split()[:2]
            vals.append(float.fromhex(hexval))
    if len(vals) != 28:
        raise ValueError(f"{POLISHED_PATH}: expected 28 coefficients, got {len(vals)}")
    return vals
