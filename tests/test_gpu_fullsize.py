"""Full-size parity of the benchmarked merge and solve workloads (on the GPU), checked
by properties that hold at any size, so no oracle run of the whole problem is needed.

* The rank-one merge of Sec. 2.2 at N = 16384 (poles i/N, rho = 1, random unit z,
  random orthogonal Q1, Q2), through the FP64-MFMA, HSS and split-precision paths.
  No pole deflates there (K = N), so the eigenvalues of D + rho z z^T interlace the
  sorted poles d and the secular function f(x) = 1 + rho sum_i z_i^2 / (d_i - x)
  increases from -inf to +inf between consecutive poles.  Hence the number of
  eigenvalues below a non-pole x is j - 1 + [f(x) > 0], j = #{d_i < x} >= 1 (and 0
  when j = 0).  It is checked at lambda_k -+ 1e-13 ||A|| for sampled k.  The
  eigenvectors are checked by orthogonality and by the residual of
  A = diag(Q1, Q2) (D + rho z z^T) diag(Q1, Q2)^T, evaluated on the GPU.
* The 1-2-1 Toeplitz solve at n = 16383 (top merge K = n) through the FP64 and HSS
  paths, against the closed form lambda_k = 2 + 2 cos(k pi/(n+1)) (all k) and
  v_k(j) = sqrt(2/(n+1)) sin(j k pi/(n+1)) (sampled well-separated k).
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

N = 16384


@pytest.fixture(scope="module")
def P():
    import paper_1612_07526_amd as P
    P.load()
    return P


@pytest.fixture(scope="module")
def s3():
    return W.fig3_merge(N, seed=0, with_q=True)


def _orth(Q):
    Qc = Q.contiguous()
    G = Qc.T @ Qc
    G.diagonal().sub_(1.0)
    v = G.abs().max().item()
    del G
    return v


def _count_below(ds, zs, rho, x):
    j = int(np.searchsorted(ds, x, side="left"))
    if j == 0:
        return 0
    f = 1.0 + rho * np.sum(zs * zs / (ds - x))
    return j - 1 + (1 if f > 0 else 0)


@pytest.mark.parametrize("mode", ["fp64", "hss", "split"])
def test_s3_merge_full_size(P, s3, mode):
    D, z, rho, Q1, Q2 = s3
    o = {"fp64": P.opts(gemm_mode=P.GEMM_FP64), "hss": P.opts(gemm_mode=P.GEMM_HSS, hss_min_K=4096),
         "split": P.opts(gemm_mode=P.GEMM_SPLIT)}[mode]
    dev = "cuda"
    Q1t = torch.tensor(Q1, device=dev)
    Q2t = torch.tensor(Q2, device=dev)
    lam, Q, work = P.merge(D, z, rho, Q1t, Q2t, o=o, return_work=True)
    st = P.merge_stats(work)
    assert st[0] == N  # no deflation
    assert st[6] == {"fp64": 0, "hss": 2, "split": 1}[mode]
    del work
    lam_h = lam.cpu().numpy()
    assert np.all(np.diff(lam_h) > 0)
    nrm = np.abs(lam_h).max()
    order = np.argsort(D, kind="stable")
    ds, zs = D[order], z[order]
    delta = 1e-13 * nrm
    for k in np.random.default_rng(1).choice(N, 48, replace=False):
        assert _count_below(ds, zs, rho, lam_h[k] - delta) <= k
        assert _count_below(ds, zs, rho, lam_h[k] + delta) >= k + 1
    # eigenvectors: orthogonality and residual of the assembled matrix
    Qd = Q.contiguous()  # (N, N), column k = eigenvector k
    orth_tol, res_tol = (1e-11, 1e-12) if mode == "split" else (1e-12, 1e-13)
    assert _orth(Qd) <= orth_tol
    n1 = Q1.shape[0]
    Y = torch.empty_like(Qd)
    Y[:n1] = Q1t.T @ Qd[:n1]
    Y[n1:] = Q2t.T @ Qd[n1:]
    Dt = torch.tensor(D, device=dev)
    zt = torch.tensor(z, device=dev)
    Wm = Dt[:, None] * Y + rho * zt[:, None] * (zt @ Y)[None, :]
    del Y
    R = torch.empty_like(Qd)
    R[:n1] = Q1t @ Wm[:n1]
    R[n1:] = Q2t @ Wm[n1:]
    del Wm
    R -= Qd * lam[None, :]
    res = (torch.linalg.norm(R) / (N * nrm)).item()
    assert res <= res_tol, res


@pytest.mark.parametrize("mode", ["fp64", "hss"])
def test_toeplitz_16383_full_size(P, mode):
    n = 16383
    d, e = W.toeplitz_121(n, 1.0)
    o = P.opts(gemm_mode=P.GEMM_FP64) if mode == "fp64" else P.opts(gemm_mode=P.GEMM_HSS)
    lam, Q, work = P.stedc(d, e, o=o, return_work=True)
    st = P.merge_stats(work)
    assert st[0] == n and st[6] == (2 if mode == "hss" else 0)  # root merge: no deflation
    del work
    k = np.arange(1, n + 1)
    lam_exact = (2.0 + 2.0 * np.cos(k * np.pi / (n + 1)))[::-1]  # ascending; column k <-> index n+1-k
    lam_h = lam.cpu().numpy()
    assert np.abs(lam_h - lam_exact).max() <= 1e-13 * 4.0
    # sampled columns against the sine eigenvectors, each within its gap bound
    # factor * max(1e-14 / gap_rel, 1e-13) (factor 10 for the HSS product)
    gaps = np.minimum(np.diff(lam_exact, prepend=-np.inf), np.diff(lam_exact, append=np.inf))
    pick = np.random.default_rng(2).choice(n, 48, replace=False)
    Qs = Q[:, torch.tensor(pick, device=Q.device)].cpu().numpy()
    j = np.arange(1, n + 1)
    factor = 10.0 if mode == "hss" else 1.0
    for c, idx in enumerate(pick):
        kk = n - idx  # ascending index idx holds the closed-form mode k = n - idx
        v = np.sqrt(2.0 / (n + 1)) * np.sin(j * kk * np.pi / (n + 1))
        q = Qs[:, c] * np.sign(np.dot(Qs[:, c], v))
        bound = factor * max(1e-14 / (gaps[idx] / 4.0), 1e-13)
        assert np.abs(q - v).max() <= bound, (idx, np.abs(q - v).max(), bound)
    Qd = Q.contiguous()
    assert _orth(Qd) <= 1e-12
    dt = torch.tensor(d, device=Qd.device)
    et = torch.tensor(e, device=Qd.device)
    R = dt[:, None] * Qd - Qd * lam[None, :]
    R[:-1] += et[:, None] * Qd[1:]
    R[1:] += et[:, None] * Qd[:-1]
    assert (torch.linalg.norm(R) / (n * 4.0)).item() <= 1e-13
