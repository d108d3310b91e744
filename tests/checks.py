"""Independent checks used by the tests (never by the library or the oracle).

Everything here is a property of the *answer*, computed from the definition of
a symmetric tridiagonal eigen-decomposition: residuals, orthogonality, Sturm
counts, closed-form spectra, sign normalisation.
"""
from __future__ import annotations

import numpy as np

U = 2.0 ** -53


def tri_dense(d, e):
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


def tri_matvec(d, e, Q):
    """T @ Q for the tridiagonal (d, e) without forming T."""
    Q = np.asarray(Q)
    R = d[:, None] * Q
    if e.size:
        R[:-1] += e[:, None] * Q[1:]
        R[1:] += e[:, None] * Q[:-1]
    return R


def tnorm(d, e):
    """2-norm of T via its extreme eigenvalues bound: max row sum (an upper bound within 3x)."""
    d = np.abs(np.asarray(d, dtype=np.float64))
    e = np.abs(np.asarray(e, dtype=np.float64))
    r = d.copy()
    if e.size:
        r[:-1] += e
        r[1:] += e
    return float(r.max()) if r.size else 0.0


def residual(d, e, lam, Q):
    """||T Q - Q Lambda||_F / (n ||T||), with ||T|| = max |lambda| (the 2-norm of the
    symmetric T, given by its computed eigenvalues; not the larger max row sum)."""
    n = len(d)
    if n == 0:
        return 0.0
    lam = np.asarray(lam)
    R = tri_matvec(np.asarray(d), np.asarray(e), Q) - Q * lam[None, :]
    return float(np.linalg.norm(R) / (n * max(float(np.abs(lam).max()), 1e-300)))


def vec_tol(gap_rel):
    """Bound on the entrywise difference of two computed unit eigenvectors whose
    eigenvalue is separated from the rest of the spectrum by gap_rel * ||T||.

    Each solver returns an exact eigenvector of some T + E; an isolated eigenvector moves
    by at most ||E|| / gap under such a perturbation (Davis-Kahan sin-theta), so two
    solutions with ||E|| <= 45 u ||T|| each (u = 2^-53; the per-column residuals of the
    solves tested are a few u ||T||) differ by at most 1e-14 / gap_rel: 1e-11 at
    gap_rel = 1e-3."""
    return 1e-14 / gap_rel


def orth(Q):
    """||Q^T Q - I||_max."""
    n = Q.shape[1]
    return float(np.abs(Q.T @ Q - np.eye(n)).max()) if n else 0.0


def sturm_count(d, e, x):
    """Number of eigenvalues of T strictly less than x (LDL^T inertia, Sylvester)."""
    cnt = 0
    q = d[0] - x
    if q < 0:
        cnt += 1
    for i in range(1, len(d)):
        if q == 0.0:
            q = 1e-300
        q = (d[i] - x) - e[i - 1] ** 2 / q
        if q < 0:
            cnt += 1
    return cnt


def canon(Q):
    """Sign-normalise columns: the entry of largest magnitude (lowest index on ties) is positive."""
    Q = np.array(Q, dtype=np.float64, copy=True)
    if Q.size == 0:
        return Q
    idx = np.argmax(np.abs(Q), axis=0)
    s = np.sign(Q[idx, np.arange(Q.shape[1])])
    s[s == 0] = 1.0
    return Q * s[None, :]


def align(Q, Qref):
    """Flip columns of Q to best match Qref (for sign-ambiguous eigenvectors)."""
    s = np.sign(np.sum(Q * Qref, axis=0))
    s[s == 0] = 1.0
    return Q * s[None, :]


def isolated_columns(lam, gap_tol):
    """Mask of eigenvalues separated from both neighbours by more than gap_tol."""
    lam = np.asarray(lam)
    n = lam.size
    ok = np.ones(n, dtype=bool)
    if n > 1:
        g = np.diff(lam)
        ok[:-1] &= g > gap_tol
        ok[1:] &= g > gap_tol
    return ok


def toeplitz_121_exact(n, off=1.0):
    """Eigenpairs of tridiag(off, 2, off), off = +-1, ascending.

    tridiag(-1, 2, -1): lambda_k = 2 - 2 cos(k pi/(n+1)), v_k(j) = sqrt(2/(n+1)) sin(j k pi/(n+1)).
    tridiag(+1, 2, +1): lambda = 2 + 2 cos(k pi/(n+1)) with the same v_k, i.e. the order of k reverses.
    """
    k = np.arange(1, n + 1)
    j = np.arange(1, n + 1)
    V = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, k) * np.pi / (n + 1))
    if off < 0:
        lam = 2.0 - 2.0 * np.cos(k * np.pi / (n + 1))
    else:
        lam = (2.0 + 2.0 * np.cos(k * np.pi / (n + 1)))[::-1]
        V = V[:, ::-1]
    return lam, V


def column_gaps(lam):
    """Distance of each eigenvalue to its nearest neighbour (inf for n = 1)."""
    lam = np.asarray(lam, dtype=np.float64)
    g = np.full(lam.size, np.inf)
    if lam.size > 1:
        dl = np.diff(lam)
        g[1:] = np.minimum(g[1:], dl)
        g[:-1] = np.minimum(g[:-1], dl)
    return g


def vector_error_ratio(Q, Qref, lref, factor=1.0, max_bound=1e-3):
    """max over columns of |sign-aligned Q(:, k) - Qref(:, k)|_max / bound_k with
    bound_k = factor * max(vec_tol(gap_k), 1e-13), gap_k the relative gap of lref[k].  The
    floor 1e-13 covers the gap-independent rounding of the update product (an entry of
    X Uhat sums up to K ~ 10^3 products of unit-norm rows and columns: K u ~ 1e-13).
    factor loosens the bound for update paths with an error of their own (HSS compression,
    split precision).  Columns whose bound exceeds max_bound (a tight cluster, where the
    vectors are not individually determined) are skipped.
    Returns (ratio, number of columns compared); the check passes when ratio <= 1."""
    Q = np.asarray(Q)
    Qref = np.asarray(Qref)
    nrm = max(float(np.abs(lref).max()), 1e-300)
    bound = factor * np.maximum(1e-14 / np.maximum(column_gaps(lref) / nrm, 1e-300), 1e-13)
    use = bound <= max_bound
    if not use.any():
        return 0.0, 0
    diff = np.abs(align(Q[:, use], Qref[:, use]) - Qref[:, use]).max(axis=0)
    return float((diff / bound[use]).max()), int(use.sum())
