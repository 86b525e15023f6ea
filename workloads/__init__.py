"""Seeded synthetic inputs for the truncated Neumann series workloads.

This module is the only code shared by the oracle and the GPU side.  It builds
input matrices and nothing else: no series, kernel or product of the method is
computed here.  All generation is host float64 NumPy from
``numpy.random.default_rng(seed)``.

The paper's random model is A = alpha * Omega D Omega^T with Omega orthogonal
and D diagonal in [-1, 1] (Sec. 6, setup); the distributions of Omega and D
are not stated, so the generators below fix them: Omega from the QR factor of
a Gaussian matrix, eigenvalues uniform on a symmetric interval.

Workloads (n is the matrix dimension, k the series length):

  small_symmetric   n=256, eigenvalues U[-0.5, 0.5], k=81, seed 1
  large_symmetric   n=4096, eigenvalues U[-0.95, 0.95], k=729, seed 2
  gaussian_rho      n=8192, N(0,1)/sqrt(n) rescaled to a power-iteration
                    spectral-radius estimate of 0.99 (0.95 for the
                    convergent variant), k=3375, seed 3
  precision_sym     n=8192, eigenvalues U[-0.9, 0.9], k=729, seed 4
  jacobi_batch      2048 matrices, n_i uniform on {8,...,256} (powers of two),
                    A_i = I - D^{-1} G, G = H^T H + 0.01 I, H ~ N(0,1) of shape
                    8 n_i x n_i, D = diag(G); k=81, seed 5.  The shape of a
                    MIMO-detection Jacobi iteration matrix (Sec. 1 names MIMO
                    detection as an application); no channel data is used.

The same construction at any other n is available for tests (``symmetric``,
``gaussian``, ``jacobi``), and ``dyadic`` builds sparse inputs whose low
powers are exact in every floating-point format the library computes in.
"""

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class SymmetricInput:
    A: np.ndarray          # n x n float64, A = Q diag(lam) Q^T (symmetrised)
    Q: np.ndarray          # orthogonal factor
    lam: np.ndarray        # eigenvalues
    seed: int


def symmetric(n: int, lam_max: float, seed: int) -> SymmetricInput:
    """A = Q diag(lam) Q^T, Q from QR of an N(0,1) n x n matrix, lam uniform
    on [-lam_max, lam_max].  A is symmetrised as (A + A^T)/2 so that the
    stored matrix is exactly symmetric."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    Q, _ = np.linalg.qr(G)
    lam = rng.uniform(-lam_max, lam_max, n)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    return SymmetricInput(A=A, Q=Q, lam=lam, seed=seed)


def dyadic(n: int, seed: int, terms: int = 3) -> np.ndarray:
    """A = (1/8) sum_t diag(s_t) P_t: ``terms`` random permutation matrices
    P_t with random row signs s_t = +-1.  Every entry is a multiple of 1/8 of
    magnitude at most terms/8, each row and column has at most ``terms``
    nonzeros, so ||A||_inf <= terms/8 and low powers of A stay on a coarse
    dyadic grid (A^j: multiples of 8^-j, at most terms^j of them per entry).
    A test input on which floating-point arithmetic of a few powers is exact."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    rows = np.arange(n)
    for _ in range(terms):
        perm = rng.permutation(n)
        sign = rng.choice([-1.0, 1.0], size=n)
        np.add.at(A, (rows, perm), sign / 8.0)
    return A


def cyclic(n: int, seed: int, scale: float = 0.5) -> np.ndarray:
    """A = scale * diag(s) P for P the permutation matrix of one random
    n-cycle and s random signs.  A^j is then scale^j times a signed
    permutation whose nonzeros sit where those of A^i (i < n, i != j) do
    not, so every power, and every sum of distinct powers, has one entry per
    row and column that is a signed power of ``scale``."""
    rng = np.random.default_rng(seed)
    order = rng.permutation(n)
    nxt = np.empty(n, dtype=np.int64)
    nxt[order] = np.roll(order, -1)               # one cycle through all of 0..n-1
    A = np.zeros((n, n))
    A[np.arange(n), nxt] = rng.choice([-1.0, 1.0], size=n) * scale
    return A


def power_iteration_radius(G: np.ndarray, seed: int, iters: int = 400,
                           tail: int = 200) -> float:
    """Spectral-radius estimate: ``iters`` power iterations from a seeded
    Gaussian vector, renormalised every step; the estimate is the geometric
    mean of the growth factors over the last ``tail`` steps (a complex
    dominant pair makes single-step growth oscillate)."""
    rng = np.random.default_rng(seed + 1_000_003)
    v = rng.standard_normal(G.shape[0])
    v /= np.linalg.norm(v)
    logs = []
    for i in range(iters):
        w = G @ v
        g = np.linalg.norm(w)
        v = w / g
        if i >= iters - tail:
            logs.append(np.log(g))
    return float(np.exp(np.mean(logs)))


@dataclass
class GaussianInput:
    A: np.ndarray
    rho_target: float
    rho_hat_before: float     # estimate for N(0,1)/sqrt(n) before scaling
    seed: int


def gaussian(n: int, rho: float, seed: int, iters: int = 400) -> GaussianInput:
    """Nonsymmetric A = s * N(0,1)/sqrt(n) with s chosen so that the
    power-iteration estimate of rho(A) equals ``rho``."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n)) / np.sqrt(n)
    r = power_iteration_radius(G, seed, iters=iters, tail=iters // 2)
    return GaussianInput(A=G * (rho / r), rho_target=rho, rho_hat_before=r, seed=seed)


def jacobi(n: int, rng: np.random.Generator) -> np.ndarray:
    """A = I - D^{-1} G with G = H^T H + 0.01 I, H ~ N(0,1) of shape 8n x n,
    D = diag(G): the Jacobi iteration matrix of a MIMO detection Gram system."""
    H = rng.standard_normal((8 * n, n))
    G = H.T @ H + 0.01 * np.eye(n)
    d = np.diag(G).copy()
    return np.eye(n) - G / d[:, None]


@dataclass
class BatchInput:
    mats: List[np.ndarray]
    ns: np.ndarray
    seed: int
    sizes: tuple = field(default=(8, 16, 32, 64, 128, 256))

    def packed(self, dtype=np.float32):
        """Row-major matrices back to back; returns (buffer, offsets)."""
        offs = np.zeros(len(self.mats), dtype=np.int64)
        total = 0
        for i, M in enumerate(self.mats):
            offs[i] = total
            total += M.size
        buf = np.empty(total, dtype=dtype)
        for i, M in enumerate(self.mats):
            buf[offs[i]:offs[i] + M.size] = M.ravel()
        return buf, offs


def jacobi_batch(batch: int, seed: int,
                 sizes=(8, 16, 32, 64, 128, 256)) -> BatchInput:
    """Sizes first (uniform over ``sizes``), then one matrix per size draw."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=batch)
    mats = [jacobi(int(n), rng) for n in ns]
    return BatchInput(mats=mats, ns=ns.astype(np.int32), seed=seed, sizes=tuple(sizes))


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n: int
    k: int
    seed: int
    description: str


WORKLOADS = {
    "small_symmetric": Workload("small_symmetric", 256, 81, 1,
                                "n=256 fp64, lam~U[-0.5,0.5], k=81"),
    "large_symmetric": Workload("large_symmetric", 4096, 729, 2,
                                "n=4096, lam~U[-0.95,0.95], k=729"),
    "gaussian_rho": Workload("gaussian_rho", 8192, 3375, 3,
                             "n=8192 fp32, N(0,1)/sqrt(n) scaled to rho_hat=0.99, k=3375"),
    "precision_sym": Workload("precision_sym", 8192, 729, 4,
                              "n=8192, lam~U[-0.9,0.9], k=729, split-bf16 / scaled fp16"),
    "jacobi_batch": Workload("jacobi_batch", 256, 81, 5,
                             "2048 Jacobi matrices, n in {8..256}, k=81, fp32"),
}

LAM_MAX = {"small_symmetric": 0.5, "large_symmetric": 0.95, "precision_sym": 0.9}


def make(name: str, n: Optional[int] = None, **kw):
    """Build a named workload's input (optionally at a smaller n, same recipe)."""
    w = WORKLOADS[name]
    n = w.n if n is None else n
    if name in LAM_MAX:
        return symmetric(n, LAM_MAX[name], w.seed)
    if name == "gaussian_rho":
        return gaussian(n, kw.get("rho", 0.99), w.seed)
    if name == "jacobi_batch":
        return jacobi_batch(kw.get("batch", 2048), w.seed)
    raise KeyError(name)
