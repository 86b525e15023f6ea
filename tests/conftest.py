import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def golden_rows(name):
    """Non-comment, non-empty rows of a golden fixture, split on whitespace."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


def close_report(got, ref):
    """(relative Frobenius error, largest element error over the largest
    reference element) of got against ref."""
    import numpy as np
    got = np.asarray(got, np.float64)
    d = got - ref
    return (float(np.linalg.norm(d) / np.linalg.norm(ref)),
            float(np.max(np.abs(d)) / np.max(np.abs(ref))))


def assert_close(got, ref, tol, what=""):
    """Both the relative Frobenius error and the element-wise error
    max|got - ref| / max|ref| within tol; prints both."""
    fro, elem = close_report(got, ref)
    print(f"   {what} rel fro {fro:.3e}  max elem err / max|ref| {elem:.3e}  (tol {tol:g})",
          flush=True)
    assert fro < tol, (what, fro, tol)
    assert elem < tol, (what, elem, tol)
    return fro, elem
