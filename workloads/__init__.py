"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws and lays out inputs; it holds none of the eigensolver's
arithmetic.  Every generator is deterministic in its seed (numpy PCG64 via
``default_rng``; draws happen in the order d, then e, then any further arrays).

Workloads (arXiv 1612.07526 uses no dataset; its test matrices are closed form):
  * ``toeplitz_121``  -- diagonal 2, off-diagonal +-1 (Example 2; the Toeplitz-type
    matrix of Example 3, Eq. (11), read as diagonal 2 and both off-diagonals 1);
  * ``clement``       -- zero diagonal, off-diagonals sqrt(i (N - i)) (Example 3, Eq. (9));
  * ``hermite``       -- zero diagonal, off-diagonals sqrt(i) (Example 3, Eq. (10));
  * ``sht``           -- the spherical-harmonic-transform tridiagonal of Example 4;
  * ``uniform``       -- d, e iid Uniform[-1, 1];
  * ``normal_pos``    -- d iid N(0,1), e iid Uniform[0.1, 1];
  * ``normal``        -- d, e iid N(0,1);
  * ``ramp``          -- d_i = 4 i / n + Uniform[-0.01, 0.01] (i = 1..n), e iid Uniform[0.1, 0.5];
  * ``batch_sizes``   -- sizes iid Uniform{32..1024};
  * ``fig3_merge``    -- the rank-one merge of Sec. 2.2 (Fig. 3): poles i/N, rho = 1, a random
    unit z, and random orthogonal Q1, Q2;
  * ``example1``      -- the two dense Toeplitz test matrices of Example 1.
"""
from __future__ import annotations

import math

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def toeplitz_121(n: int, off: float = 1.0):
    """Diagonal 2, off-diagonal ``off`` (use -1.0 for the d_i = 2, e_i = -1 variant)."""
    return np.full(n, 2.0), np.full(max(n - 1, 0), float(off))


def clement(n: int):
    i = np.arange(1, n, dtype=np.float64)
    return np.zeros(n), np.sqrt(i * (n - i))


def hermite(n: int):
    return np.zeros(n), np.sqrt(np.arange(1, n, dtype=np.float64))


def sht(n: int, m: int | None = None):
    """Tridiagonal of Example 4 with j = 0..n-1: diagonal d_{m+2j}, off-diagonal c_{m+2j}."""
    if m is None:
        m = n
    l_diag = m + 2 * np.arange(n, dtype=np.float64)
    dl = (2 * l_diag * (l_diag + 1) - 2 * m * m - 1) / ((2 * l_diag - 1) * (2 * l_diag + 3))
    l_off = m + 2 * np.arange(n - 1, dtype=np.float64)
    num = (l_off - m + 1) * (l_off - m + 2) * (l_off + m + 1) * (l_off + m + 2)
    den = (2 * l_off + 1) * (2 * l_off + 3) ** 2 * (2 * l_off + 5)
    return dl, np.sqrt(num / den)


def uniform(n: int, seed: int = 0):
    g = rng(seed)
    d = g.uniform(-1.0, 1.0, n)
    e = g.uniform(-1.0, 1.0, max(n - 1, 0))
    return d, e


def normal_pos(n: int, seed: int = 0):
    g = rng(seed)
    d = g.standard_normal(n)
    e = g.uniform(0.1, 1.0, max(n - 1, 0))
    return d, e


def normal(n: int, seed: int = 0):
    g = rng(seed)
    d = g.standard_normal(n)
    e = g.standard_normal(max(n - 1, 0))
    return d, e


def ramp(n: int, seed: int = 0):
    g = rng(seed)
    d = 4.0 * np.arange(1, n + 1, dtype=np.float64) / n + g.uniform(-0.01, 0.01, n)
    e = g.uniform(0.1, 0.5, max(n - 1, 0))
    return d, e


def ramp_batch(batch: int, n: int, seed: int = 0):
    """``batch`` ramp matrices plus loss weights w ~ N(0,1) (n) and G ~ N(0,1) (n x n) each."""
    g = rng(seed)
    d = 4.0 * np.arange(1, n + 1, dtype=np.float64)[None, :] / n + g.uniform(-0.01, 0.01, (batch, n))
    e = g.uniform(0.1, 0.5, (batch, max(n - 1, 0)))
    w = g.standard_normal((batch, n))
    G = g.standard_normal((batch, n, n))
    return d, e, w, G


def batch_sizes(count: int = 4096, lo: int = 32, hi: int = 1024, seed: int = 0):
    return rng(seed).integers(lo, hi + 1, count)


def normal_batch(sizes, seed: int = 0):
    """Packed d and e for a batch: sizes drawn first (``batch_sizes``), then d, e per matrix."""
    g = rng(seed + 1)
    ds, es = [], []
    for nb in sizes:
        ds.append(g.standard_normal(int(nb)))
        es.append(g.standard_normal(max(int(nb) - 1, 0)))
    return ds, es


def random_orthogonal(n: int, g: np.random.Generator):
    if n == 0:
        return np.zeros((0, 0))
    A = g.standard_normal((n, n))
    Q, R = np.linalg.qr(A)
    return Q * np.sign(np.diag(R))[None, :]


def fig3_merge(N: int, seed: int = 0, with_q: bool | str = True):
    """Rank-one merge of Sec. 2.2: d_i = i/N (i = 1..N), rho = 1, z a random unit vector.

    Split in halves n1 = N//2, n2 = N - n1; Q1, Q2 random orthogonal (QR of Gaussian).
    with_q="gaussian" returns the two Gaussian matrices instead, for a caller that
    orthonormalises them elsewhere (large N, where a host QR takes minutes).
    """
    g = rng(seed)
    D = np.arange(1, N + 1, dtype=np.float64) / N
    z = g.standard_normal(N)
    z /= np.linalg.norm(z)
    n1 = N // 2
    if with_q == "gaussian":
        Q1 = g.standard_normal((n1, n1))
        Q2 = g.standard_normal((N - n1, N - n1))
    elif with_q:
        Q1 = random_orthogonal(n1, g)
        Q2 = random_orthogonal(N - n1, g)
    else:
        Q1 = Q2 = None
    return D, z, 1.0, Q1, Q2


def random_merge(n1: int, n2: int, seed: int = 0, dup: int = 0, tiny: int = 0):
    """Generic merge input: ascending D1, D2 ~ N(0,1), z ~ N(0,1), rho ~ U[0.5, 2].

    ``dup`` poles of D2 are set equal to poles of D1 (forcing type-2 deflation) and
    ``tiny`` entries of z are set to 1e-20 (forcing type-1 deflation).
    """
    g = rng(seed)
    D1 = np.sort(g.standard_normal(n1))
    D2 = np.sort(g.standard_normal(n2))
    if dup and n1 and n2:
        k = min(dup, n1, n2)
        idx1 = g.choice(n1, k, replace=False)
        idx2 = g.choice(n2, k, replace=False)
        D2[idx2] = D1[idx1]
        D2 = np.sort(D2)
    z = g.standard_normal(n1 + n2)
    if tiny:
        z[g.choice(n1 + n2, min(tiny, n1 + n2), replace=False)] = 1e-20
    rho = float(g.uniform(0.5, 2.0))
    Q1 = random_orthogonal(n1, g)
    Q2 = random_orthogonal(n2, g)
    return np.concatenate([D1, D2]), z, rho, Q1, Q2


def example1(n: int, which: int = 1, dpar: float = 0.1):
    """Dense Toeplitz matrices of Example 1 (Mat1: a_ii = n^2, a_ij = i - j; Mat2: kinetic energy)."""
    i = np.arange(n, dtype=np.float64)
    diff = i[:, None] - i[None, :]
    if which == 1:
        A = diff.copy()
        np.fill_diagonal(A, float(n) ** 2)
        return A
    with np.errstate(divide="ignore"):
        A = ((-1.0) ** np.abs(diff)) / (diff ** 2 * dpar ** 2)
    np.fill_diagonal(A, math.pi ** 2 / (6 * dpar ** 2))
    return A


# Named configurations (sizes as used by the benchmark and the parity tests).
CONFIGS = {
    "toeplitz121_n2048": dict(kind="toeplitz_121", n=2048, off=-1.0),
    "uniform_n16384": dict(kind="uniform", n=16384, seed=0),
    "normalpos_n32768": dict(kind="normal_pos", n=32768, seed=0),
    "batch4096": dict(kind="batch", count=4096, seed=0),
    "ramp_b64_n4096": dict(kind="ramp_batch", batch=64, n=4096, seed=0),
}


def weak_coupling(n: int, seed: int = 0, every: int = 5):
    """d ~ N(0, 1); one off-diagonal entry in `every` ~ N(0, 1), the rest ~ 1e-18 N(0, 1):
    most z entries fall below the deflation tolerance at every merge (type-1 deflation)."""
    g = rng(seed)
    d = g.standard_normal(n)
    e = 1e-18 * g.standard_normal(max(n - 1, 0))
    e[::every] = g.standard_normal(len(e[::every]))
    return d, e


def glued_blocks(n: int, block: int = 7, glue: float = 1e-9):
    """Copies of the block tridiag(1, |c - i|, 1) (c = block // 2) joined by off-diagonal
    entries `glue`: nearly equal eigenvalues in both halves of a merge, which deflate by
    rotations between columns of Q1 and Q2 (type 2)."""
    i = np.arange(n)
    d = np.abs((block // 2) - (i % block)).astype(np.float64)
    e = np.where((np.arange(1, n) % block) == 0, glue, 1.0).astype(np.float64)
    return d, e


def tridiag(kind: str, n: int, seed: int = 0, **kw):
    if kind == "toeplitz_121":
        return toeplitz_121(n, kw.get("off", 1.0))
    if kind == "clement":
        return clement(n)
    if kind == "hermite":
        return hermite(n)
    if kind == "sht":
        return sht(n, kw.get("m"))
    if kind == "uniform":
        return uniform(n, seed)
    if kind == "normal_pos":
        return normal_pos(n, seed)
    if kind == "normal":
        return normal(n, seed)
    if kind == "ramp":
        return ramp(n, seed)
    if kind == "weak_coupling":
        return weak_coupling(n, seed)
    if kind == "glued":
        return glued_blocks(n)
    raise ValueError(kind)
