"""The two alternative merge-update paths against the CPU oracle, on the GPU.

HSS (Sec. 2.2, Algorithm 1): Uhat compressed by randomized sampling and
interpolative decompositions with relative tolerance hss_rel_tol = 1e-14, the
product applied in HSS form.  The result must meet the same bounds as the FP64
path (the compression error is below the FP64 rounding of the product).

Split precision: BF16 slices on the matrix cores with FP32 accumulation and FP64
recombination; bounds loosened by 10x (orthogonality 1e-11, residual 1e-12).
Eigenvalues do not depend on the update product and keep the FP64 bound.
"""
import numpy as np
import pytest
import torch

import workloads as W
from checks import align, isolated_columns, orth, residual, toeplitz_121_exact, vec_tol, vector_error_ratio

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1612_07526_amd as P
    P.load()
    return P


def _np(t):
    return t.detach().cpu().numpy()


# The HSS product adds the compression error (entries of Uhat truncated at about
# hss_rel_tol sqrt(d) ~ 1e-13, d = 192 samples) to every update column, independent of
# the eigenvalue gap: eigenvector bounds are 10x those of the FP64 path.
HSS_FACTOR = 10.0


def _hss(P, min_k, leaf=128, d=192):
    return P.opts(gemm_mode=P.GEMM_HSS, hss_min_K=min_k, hss_leaf=leaf, hss_samples=d, hss_samples_inc=64)


def _merge_check(P, orc, D, z, rho, Q1, Q2, o, orth_tol, res_tol, vec_factor=1.0):
    lref, Qref, st_ref = orc.merge(D, z, rho, Q1, Q2)
    lam, Q, work = P.merge(D, z, rho, torch.tensor(Q1), torch.tensor(Q2), o=o, return_work=True)
    st = P.merge_stats(work)
    lam, Q = _np(lam), _np(Q)
    n1 = Q1.shape[0]
    m = D.size
    Qb = np.zeros((m, m))
    Qb[:n1, :n1] = Q1
    Qb[n1:, n1:] = Q2
    A = Qb @ (np.diag(D) + rho * np.outer(z, z)) @ Qb.T
    nrm = np.abs(lref).max()
    assert np.abs(lam - lref).max() <= 1e-13 * nrm
    assert orth(Q) <= orth_tol
    assert np.linalg.norm(A @ Q - Q * lam) / (m * nrm) <= res_tol
    ratio, ncols = vector_error_ratio(Q, Qref, lref, factor=vec_factor)
    assert ratio <= 1.0, f"eigenvector error {ratio:.2f} x the gap bound ({ncols} columns)"
    assert list(st[:6]) == list(st_ref[:6])
    return st


# ---------------------------------------------------------------- HSS


@pytest.mark.parametrize("N,leaf,seed", [(600, 64, 0), (2048, 128, 1), (3001, 256, 2)])
def test_hss_merge_fig3(P, orc, N, leaf, seed):
    # the rank-one merge of Sec. 2.2: poles i/N, rho = 1, random unit z, no deflation
    D, z, rho, Q1, Q2 = W.fig3_merge(N, seed=seed)
    st = _merge_check(P, orc, D, z, rho, Q1, Q2, _hss(P, 256, leaf), 1e-12, 1e-13, HSS_FACTOR)
    assert st[6] == 2 and 0 < st[7] < 192  # HSS path taken, ranks found below the sample count


def test_hss_merge_with_deflation(P, orc):
    D, z, rho, Q1, Q2 = W.random_merge(700, 650, seed=9, dup=50, tiny=40)
    st = _merge_check(P, orc, D, z, rho, Q1, Q2, _hss(P, 256, 128), 1e-12, 1e-13, HSS_FACTOR)
    assert st[6] == 2


def test_hss_below_threshold_is_plain(P, orc):
    D, z, rho, Q1, Q2 = W.random_merge(100, 90, seed=3)
    st = _merge_check(P, orc, D, z, rho, Q1, Q2, _hss(P, 4096), 1e-12, 1e-13)
    assert st[6] == 0


@pytest.mark.parametrize("n", [2047, 4095])
def test_hss_stedc_toeplitz_odd(P, n):
    # odd order: the halves differ, no pole deflates at the top merge (K = n)
    d, e = W.toeplitz_121(n, 1.0)
    lam, Q, work = P.stedc(d, e, o=_hss(P, 1024), return_work=True)
    st = P.merge_stats(work)
    assert st[0] == n and st[6] == 2
    lr, Vr = toeplitz_121_exact(n, 1.0)
    lam, Q = _np(lam), _np(Q)
    assert np.abs(lam - lr).max() <= 1e-13 * 4
    assert orth(Q) <= 1e-12
    assert residual(d, e, lam, Q) <= 1e-13
    ratio, ncols = vector_error_ratio(Q, Vr, lr)
    assert ratio <= 1.0 and ncols == n, (ratio, ncols)


@pytest.mark.parametrize("gen,n", [("clement", 2047), ("hermite", 2048)])
def test_hss_stedc_example3(P, orc, gen, n):
    d, e = W.tridiag(gen, n)
    lref, _, _ = orc.stedc(d, e)
    lam, Q = P.stedc(d, e, o=_hss(P, 512))
    lam, Q = _np(lam), _np(Q)
    assert np.abs(lam - lref).max() <= 1e-13 * np.abs(lref).max()
    assert orth(Q) <= 1e-12
    assert residual(d, e, lam, Q) <= 1e-13


# ---------------------------------------------------------------- split precision


@pytest.mark.parametrize("n1,n2,dup,tiny,seed", [(3, 2, 0, 0, 1), (64, 64, 0, 9, 4), (127, 129, 20, 20, 5),
                                                 (300, 513, 0, 0, 8), (700, 650, 50, 40, 9)])
def test_split_merge(P, orc, n1, n2, dup, tiny, seed):
    D, z, rho, Q1, Q2 = W.random_merge(n1, n2, seed=seed, dup=dup, tiny=tiny)
    st = _merge_check(P, orc, D, z, rho, Q1, Q2, P.opts(gemm_mode=P.GEMM_SPLIT), 1e-11, 1e-12, 10.0)
    assert st[6] == 1


def test_split_fig3(P, orc):
    D, z, rho, Q1, Q2 = W.fig3_merge(2000, seed=4)
    _merge_check(P, orc, D, z, rho, Q1, Q2, P.opts(gemm_mode=P.GEMM_SPLIT), 1e-11, 1e-12, 10.0)


def test_split_error_shrinks_with_slices(P, orc):
    D, z, rho, Q1, Q2 = W.fig3_merge(600, seed=5)
    lref, Qref, _ = orc.merge(D, z, rho, Q1, Q2)
    errs = []
    for s in (3, 5, 7):
        lam, Q = P.merge(D, z, rho, torch.tensor(Q1), torch.tensor(Q2),
                         o=P.opts(gemm_mode=P.GEMM_SPLIT, split_slices=s))
        errs.append(np.abs(align(_np(Q), Qref) - Qref).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] < 2.0 ** (-8 * 3 + 12)  # about 2^-8s relative per entry, times growth with K


@pytest.mark.parametrize("gen,n,seed", [("normal_pos", 2048, 0), ("toeplitz_121", 2047, 0)])
def test_split_stedc(P, orc, gen, n, seed):
    d, e = W.tridiag(gen, n, seed)
    lref, _, _ = orc.stedc(d, e)
    lam, Q = P.stedc(d, e, o=P.opts(gemm_mode=P.GEMM_SPLIT))
    lam, Q = _np(lam), _np(Q)
    assert np.abs(lam - lref).max() <= 1e-13 * np.abs(lref).max()
    assert orth(Q) <= 1e-11
    assert residual(d, e, lam, Q) <= 1e-12


def test_split_stedc_full_size_32768(P):
    # the split-precision workload at its full size: n = 32768, d ~ N(0,1), e ~ U[0.1, 1];
    # eigenvalues checked by Sturm counts at sampled points, orthogonality and
    # residual of the full Q on the GPU
    from checks import sturm_count
    n = 32768
    d, e = W.normal_pos(n, 0)
    lam, Q = P.stedc(d, e, o=P.opts(gemm_mode=P.GEMM_SPLIT))
    lam_h = _np(lam)
    nrm = np.abs(lam_h).max()
    for k in np.random.default_rng(0).choice(n, 24, replace=False):
        delta = 1e-12 * nrm
        lo, hi = sturm_count(d, e, lam_h[k] - delta), sturm_count(d, e, lam_h[k] + delta)
        assert lo <= k < hi
    Qd = Q.contiguous()
    G = Qd.T @ Qd
    G.diagonal().sub_(1.0)
    assert G.abs().max().item() <= 1e-11
    del G
    dt = torch.tensor(d, device=Qd.device)
    et = torch.tensor(e, device=Qd.device)
    R = dt[:, None] * Qd - Qd * lam[None, :]
    R[:-1] += et[:, None] * Qd[1:]
    R[1:] += et[:, None] * Qd[:-1]
    assert (torch.linalg.norm(R) / (n * nrm)).item() <= 1e-12
