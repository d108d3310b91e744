"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each test checks an oracle routine against something other than itself:
closed-form spectra (Toeplitz 1-2-1 of Example 2/3, Clement Eq. (9), Hermite
Eq. (10)), Sturm counts, trace invariants, LAPACK through numpy/scipy (the
library special case of an exact eigensolver), dense brute force on small
inputs, interlacing, and first-order perturbation theory for the adjoint.
"""
import numpy as np
import pytest
import scipy.linalg

import workloads as W
from checks import (U, align, isolated_columns, orth, residual, sturm_count, tnorm,
                    toeplitz_121_exact, tri_dense)

# ---------------------------------------------------------------- Jacobi leaf


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 32, 64])
def test_jacobi_vs_lapack(orc, n):
    g = np.random.default_rng(n)
    A = g.standard_normal((n, n))
    A = A + A.T
    w, V = orc.jacobi(A)
    wr = np.linalg.eigvalsh(A)
    nrm = np.abs(wr).max()
    assert np.abs(w - wr).max() <= 1e-13 * nrm
    assert orth(V) <= 1e-13
    assert np.linalg.norm(A @ V - V * w) <= 1e-13 * n * nrm


def test_jacobi_diagonal_and_repeated(orc):
    A = np.diag([3.0, -1.0, 3.0, 0.0])
    w, V = orc.jacobi(A)
    assert np.array_equal(w, [-1.0, 0.0, 3.0, 3.0])
    assert orth(V) == 0.0


# ---------------------------------------------------------------- secular roots


def _dpr(K, seed, rho=1.3):
    g = np.random.default_rng(seed)
    d = np.sort(g.standard_normal(K))
    z = g.standard_normal(K)
    z /= np.linalg.norm(z)
    return d, z, rho


def test_secular_K1_closed_form(orc):
    d, z, rho = np.array([0.25]), np.array([-0.6]), 2.0
    o, tau = orc.secular(d, z, rho)
    assert o[0] == 0
    assert abs(tau[0] - rho * 0.36) <= 4 * U * rho * 0.36


def test_secular_K2_closed_form(orc):
    d = np.array([-0.5, 1.0])
    z = np.array([0.6, 0.8])
    rho = 1.5
    o, tau = orc.secular(d, z, rho)
    lam = d[o] + tau
    # eigenvalues of [[d1 + rho z1^2, rho z1 z2], [rho z1 z2, d2 + rho z2^2]] by the quadratic formula
    a, c, b = d[0] + rho * z[0] ** 2, d[1] + rho * z[1] ** 2, rho * z[0] * z[1]
    m, r = 0.5 * (a + c), np.hypot(0.5 * (a - c), b)
    assert np.allclose(lam, [m - r, m + r], rtol=0, atol=1e-15)


@pytest.mark.parametrize("K,seed", [(3, 0), (17, 1), (64, 2), (300, 3)])
def test_secular_vs_dense(orc, K, seed):
    d, z, rho = _dpr(K, seed)
    o, tau = orc.secular(d, z, rho)
    lam = d[o] + tau
    ref = np.linalg.eigvalsh(np.diag(d) + rho * np.outer(z, z))
    assert np.abs(lam - ref).max() <= 1e-14 * (np.abs(d).max() + rho)
    # strict interlacing d_j < lambda_j < d_{j+1}, last root below d_K + rho |z|^2
    assert np.all(lam > d)
    assert np.all(lam[:-1] < d[1:])
    assert lam[-1] <= d[-1] + rho * (1 + 4 * U)
    # trace invariant
    assert abs(lam.sum() - (d.sum() + rho)) <= 1e-13 * K * (np.abs(d).max() + rho)
    # origin is the nearer pole of the bracket
    for j in range(K - 1):
        assert o[j] in (j, j + 1)
        assert abs(tau[j]) <= 0.5 * (d[j + 1] - d[j]) * (1 + 4 * U)


def test_secular_close_poles(orc):
    # poles 1e-12 apart: tau must resolve the gap with full relative accuracy
    d = np.array([0.0, 1e-12, 1.0, 2.0])
    z = np.array([0.5, 0.5, 0.5, 0.5])
    o, tau = orc.secular(d, z, 1.0)
    assert o[0] in (0, 1)
    lam0 = d[o[0]] + tau[0]
    assert 0.0 < lam0 < 1e-12
    # the root satisfies the secular equation evaluated in the (o, tau) form
    f = 1 + np.sum(z ** 2 / ((d - d[o[0]]) - tau[0]))
    dfdt = np.sum(z ** 2 / ((d - d[o[0]]) - tau[0]) ** 2)
    assert abs(f) / dfdt <= 1e-26


# ---------------------------------------------------------------- Loewner + eigenvectors


@pytest.mark.parametrize("K,seed", [(2, 4), (9, 5), (80, 6), (400, 7)])
def test_lowner_and_uhat(orc, K, seed):
    d, z, rho = _dpr(K, seed)
    o, tau = orc.secular(d, z, rho)
    lam = d[o] + tau
    zh = orc.lowner(d, rho, o, tau, z)
    # zhat reproduces z (the computed lambdas are near-exact eigenvalues of D + rho z z^T)
    assert np.abs(zh - z).max() <= 50 * K * U
    assert np.all(np.sign(zh) == np.sign(z))
    # lambda are eigenvalues of D + rho zhat zhat^T
    ref = np.linalg.eigvalsh(np.diag(d) + rho * np.outer(zh, zh))
    assert np.abs(lam - ref).max() <= 1e-14 * (np.abs(d).max() + rho)
    Uh = orc.uhat(d, o, tau, zh)
    assert orth(Uh) <= 20 * K * U
    M = np.diag(d) + rho * np.outer(zh, zh)
    assert np.linalg.norm(M @ Uh - Uh * lam) <= 10 * K * U * (np.abs(d).max() + rho)
    # each column is (D - lambda_j)^{-1} zhat up to scale
    j = K // 2
    v = zh / (d - lam[j])
    v /= np.linalg.norm(v)
    assert np.abs(np.abs(Uh[:, j]) - np.abs(v)).max() <= 1e-10


# ---------------------------------------------------------------- merge (Eq. (3)-(6))


def _assembled(D, z, rho, Q1, Q2):
    n1 = Q1.shape[0]
    m = D.size
    Qb = np.zeros((m, m))
    Qb[:n1, :n1] = Q1
    Qb[n1:, n1:] = Q2
    return Qb @ (np.diag(D) + rho * np.outer(z, z)) @ Qb.T


@pytest.mark.parametrize("n1,n2,dup,tiny,seed", [
    (1, 1, 0, 0, 0), (5, 3, 0, 0, 1), (16, 16, 0, 0, 2), (20, 13, 4, 0, 3), (31, 40, 0, 9, 4),
    (64, 64, 10, 10, 5), (100, 57, 0, 0, 6)])
def test_merge_vs_dense(orc, n1, n2, dup, tiny, seed):
    D, z, rho, Q1, Q2 = W.random_merge(n1, n2, seed=seed, dup=dup, tiny=tiny)
    lam, Q, st = orc.merge(D, z, rho, Q1, Q2)
    A = _assembled(D, z, rho, Q1, Q2)
    wr, Vr = np.linalg.eigh(A)
    nrm = np.abs(wr).max()
    m = n1 + n2
    assert np.all(np.diff(lam) >= 0)
    assert np.abs(lam - wr).max() <= 1e-13 * nrm
    assert orth(Q) <= 1e-12
    assert np.linalg.norm(A @ Q - Q * lam) / (m * nrm) <= 1e-13
    iso = isolated_columns(wr, 1e-6 * nrm)
    Qa = align(Q, Vr)
    assert np.abs(Qa[:, iso] - Vr[:, iso]).max() <= 1e-9
    K, k1, k2, k3, nt1, nt2 = st[:6]
    assert K == k1 + k2 + k3 and K + nt1 + nt2 == m
    # exactly equal poles always deflate one of the pair (by rotation unless a tiny z got there
    # first); z entries of 1e-20 always deflate
    assert nt1 + nt2 >= min(dup, n1, n2)
    if not tiny:
        assert nt2 >= min(dup, n1, n2)
    assert nt1 >= min(tiny, m)


def test_merge_exact_counts(orc):
    # poles of D2 equal to poles of D1 -> exactly one rotation per pair, no other deflation
    g = np.random.default_rng(11)
    D1 = np.sort(g.uniform(0, 1, 6))
    D = np.concatenate([D1, D1])
    z = g.uniform(0.5, 1.0, 12)
    Q1 = W.random_orthogonal(6, g)
    Q2 = W.random_orthogonal(6, g)
    lam, Q, st = orc.merge(D, z, 1.0, Q1, Q2)
    assert list(st[:6]) == [6, 0, 6, 0, 0, 6]
    A = _assembled(D, z, 1.0, Q1, Q2)
    assert np.abs(lam - np.linalg.eigvalsh(A)).max() <= 1e-13 * np.abs(lam).max()


def test_merge_rho_zero_and_z_zero(orc):
    g = np.random.default_rng(12)
    D = np.concatenate([np.sort(g.standard_normal(4)), np.sort(g.standard_normal(3))])
    Q1 = W.random_orthogonal(4, g)
    Q2 = W.random_orthogonal(3, g)
    for z, rho in ((g.standard_normal(7), 0.0), (np.zeros(7), 1.0)):
        lam, Q, st = orc.merge(D, z, rho, Q1, Q2)
        assert st[0] == 0 and st[4] == 7
        assert np.array_equal(lam, np.sort(D))
        assert orth(Q) <= 1e-14


# ---------------------------------------------------------------- whole solve


@pytest.mark.parametrize("n", [1, 2, 3, 32, 33, 64, 100, 257])
@pytest.mark.parametrize("off", [1.0, -1.0])
def test_stedc_toeplitz_closed_form(orc, n, off):
    d, e = W.toeplitz_121(n, off)
    lam, Q, _ = orc.stedc(d, e)
    lr, Vr = toeplitz_121_exact(n, off)
    assert np.abs(lam - lr).max() <= 1e-13 * 4
    # all eigenvalues are simple; columns agree up to sign
    assert np.abs(align(Q, Vr) - Vr).max() <= 1e-11
    assert orth(Q) <= 1e-12
    assert residual(d, e, lam, Q) <= 1e-13


def test_stedc_toeplitz_2048_balanced_split(orc):
    # n = 2048 with leaf 32: the halves are mirror images, so each merge of size m deflates
    # exactly m/2 poles by rotation and none by a small z entry.
    d, e = W.toeplitz_121(2048, -1.0)
    lam, Q, st = orc.stedc(d, e, leaf=32)
    lr, _ = toeplitz_121_exact(2048, -1.0)
    assert np.abs(lam - lr).max() <= 1e-13 * 4
    assert list(st[:6]) == [1024, 0, 1024, 0, 0, 1024]
    assert orth(Q) <= 1e-12
    assert residual(d, e, lam, Q) <= 1e-13


@pytest.mark.parametrize("n", [2, 9, 16, 63, 200])
def test_stedc_clement(orc, n):
    d, e = W.clement(n)
    lam, Q, _ = orc.stedc(d, e)
    ref = np.arange(-(n - 1), n, 2, dtype=np.float64)
    assert np.abs(lam - ref).max() <= 1e-13 * (n - 1)
    assert orth(Q) <= 1e-12
    assert residual(d, e, lam, Q) <= 1e-13


@pytest.mark.parametrize("n", [12, 40, 90])
def test_stedc_hermite(orc, n):
    d, e = W.hermite(n)
    lam, Q, _ = orc.stedc(d, e)
    nodes, _ = np.polynomial.hermite_e.hermegauss(n)
    assert np.abs(lam - np.sort(nodes)).max() <= 1e-12 * np.abs(nodes).max()
    assert orth(Q) <= 1e-12


@pytest.mark.parametrize("gen,n,seed", [("uniform", 300, 0), ("normal_pos", 257, 1), ("normal", 500, 2),
                                        ("ramp", 400, 3)])
def test_stedc_random_vs_lapack(orc, gen, n, seed):
    d, e = W.tridiag(gen, n, seed)
    lam, Q, _ = orc.stedc(d, e)
    wr, Vr = scipy.linalg.eigh_tridiagonal(d, e)
    nrm = np.abs(wr).max()
    assert np.abs(lam - wr).max() <= 1e-13 * nrm
    assert orth(Q) <= 1e-12
    assert residual(d, e, lam, Q) <= 1e-13
    iso = isolated_columns(wr, 1e-5 * nrm)
    assert np.abs(align(Q, Vr)[:, iso] - Vr[:, iso]).max() <= 1e-8
    # trace and Frobenius invariants
    assert abs(lam.sum() - d.sum()) <= 1e-12 * n * nrm
    assert abs((lam ** 2).sum() - ((d ** 2).sum() + 2 * (e ** 2).sum())) <= 1e-12 * n * nrm ** 2


@pytest.mark.parametrize("seed", [0, 1])
def test_stedc_sturm_counts(orc, seed):
    d, e = W.normal(200, seed)
    lam, _, _ = orc.stedc(d, e)
    delta = 1e-9 * tnorm(d, e)
    gaps = np.diff(lam)
    for k in range(0, 200, 7):
        if (k > 0 and gaps[k - 1] < 4 * delta) or (k < 199 and gaps[k] < 4 * delta):
            continue
        assert sturm_count(d, e, lam[k] - delta) == k
        assert sturm_count(d, e, lam[k] + delta) == k + 1


@pytest.mark.parametrize("leaf", [1, 2, 5, 32, 64])
def test_stedc_leaf_sizes_agree(orc, leaf):
    d, e = W.uniform(150, 9)
    lam, Q, _ = orc.stedc(d, e, leaf=leaf)
    wr = np.linalg.eigvalsh(tri_dense(d, e))
    assert np.abs(lam - wr).max() <= 1e-13 * np.abs(wr).max()
    assert orth(Q) <= 1e-12
    assert residual(d, e, lam, Q) <= 1e-13


def test_stedc_decoupled_blocks(orc):
    # zero off-diagonal entries make rho = 0 at those splits: every pole deflates
    d, e = W.normal(96, 4)
    e[47] = 0.0
    e[23] = 0.0
    lam, Q, st = orc.stedc(d, e)
    assert st[0] == 0
    wr = np.linalg.eigvalsh(tri_dense(d, e))
    assert np.abs(lam - wr).max() <= 1e-13 * np.abs(wr).max()
    assert residual(d, e, lam, Q) <= 1e-13


def test_stedc_empty(orc):
    lam, Q, _ = orc.stedc(np.zeros(0), np.zeros(0))
    assert lam.size == 0 and Q.size == 0


# ---------------------------------------------------------------- adjoint


def test_adjoint_eigenvalue_part_closed_form(orc):
    # L = sum_k w_k lambda_k: d lambda_k / d d_i = Q_ik^2, d lambda_k / d e_i = 2 Q_ik Q_{i+1,k}
    d, e = W.ramp(60, 1)
    lam, Q, _ = orc.stedc(d, e)
    w = np.random.default_rng(2).standard_normal(60)
    dbar, ebar = orc.adjoint(lam, Q, w, np.zeros((60, 60)))
    assert np.allclose(dbar, (Q ** 2) @ w, atol=1e-13)
    assert np.allclose(ebar, 2 * (Q[:-1] * Q[1:]) @ w, atol=1e-13)


def _loss_canon(d, e, w, G):
    lam, V = np.linalg.eigh(tri_dense(d, e))
    from checks import canon
    V = canon(V)
    return float(w @ lam + np.sum(G * V)), V


def test_adjoint_vs_central_fd(orc):
    n = 9
    g = np.random.default_rng(5)
    d = np.arange(1, n + 1, dtype=np.float64) + g.uniform(-0.1, 0.1, n)
    e = g.uniform(0.1, 0.5, n - 1)
    w = g.standard_normal(n)
    G = g.standard_normal((n, n))
    lam, Q, _ = orc.stedc(d, e)
    from checks import canon
    Qc = canon(Q)
    dbar, ebar = orc.adjoint(lam, Qc, w, G)
    h = 1e-6
    gd = np.zeros(n)
    ge = np.zeros(n - 1)
    for i in range(n):
        dp = d.copy(); dp[i] += h
        dm = d.copy(); dm[i] -= h
        gd[i] = (_loss_canon(dp, e, w, G)[0] - _loss_canon(dm, e, w, G)[0]) / (2 * h)
    for i in range(n - 1):
        ep = e.copy(); ep[i] += h
        em = e.copy(); em[i] -= h
        ge[i] = (_loss_canon(d, ep, w, G)[0] - _loss_canon(d, em, w, G)[0]) / (2 * h)
    g_all = np.concatenate([dbar, ebar])
    fd = np.concatenate([gd, ge])
    assert np.abs(g_all - fd).max() <= 1e-6 * np.abs(fd).max()


def test_gemm_plain(orc):
    g = np.random.default_rng(3)
    A = g.standard_normal((13, 7))
    B = g.standard_normal((7, 5))
    assert np.allclose(orc.gemm(A, B), A @ B, rtol=0, atol=1e-13)
