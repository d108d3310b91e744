"""The paper's Example 1 (Table 1): HSS compression of two dense Toeplitz matrices
and the product with a dense matrix, against the plain product.

Mat1: a_ii = n^2, a_ij = i - j.  Every off-diagonal block A(I, J) (I, J disjoint
index sets) equals i 1^T - 1 j^T restricted to I x J: rank exactly 2.  Mat2: the
kinetic-energy matrix a_ii = pi^2 / (6 delta^2), a_ij = (-1)^(i-j) / ((i-j)^2
delta^2), delta = 0.1, whose off-diagonal blocks have a slowly growing numerical
rank.  These structural facts are pinned on the CPU (SVD); the GPU tests check
the HSS product C = X A against numpy's X @ A and the ranks the compression finds.
"""
import numpy as np
import pytest
import torch

import workloads as W


def _offdiag_singular_values(A, lo, hi):
    """Singular values of the HSS block row A(lo:hi, outside lo:hi)."""
    cols = np.r_[0:lo, hi:A.shape[0]]
    return np.linalg.svd(A[lo:hi][:, cols], compute_uv=False)


@pytest.mark.parametrize("n,lo,hi", [(256, 0, 64), (256, 64, 128), (400, 150, 260), (512, 256, 512)])
def test_mat1_offdiagonal_rank_is_two(n, lo, hi):
    A = W.example1(n, 1)
    s = _offdiag_singular_values(A, lo, hi)
    assert s[1] > 1e-3 * s[0]
    assert s[2] <= 1e-14 * s[0]


def test_mat2_offdiagonal_rank_moderate():
    # numerical rank at 1e-14 of Mat2's block rows: far below the block size, growing
    # slowly with it (the property the HSS compression relies on)
    A = W.example1(1024, 2)
    ranks = []
    for lo, hi in ((0, 128), (128, 256), (256, 512), (0, 512)):
        s = _offdiag_singular_values(A, lo, hi)
        ranks.append(int(np.sum(s > 1e-14 * s[0])))
    assert all(r < 0.5 * (hi - lo) for r, (lo, hi) in zip(ranks, ((0, 128), (128, 256), (256, 512), (0, 512))))
    assert ranks[3] >= ranks[0]


@pytest.fixture(scope="module")
def P():
    import paper_1612_07526_amd as P
    P.load()
    return P


def _colmajor(M):
    """A device tensor with column-major storage holding M (numpy)."""
    return torch.tensor(np.ascontiguousarray(M.T), device="cuda").t()


@pytest.mark.gpu
@pytest.mark.parametrize("which,n,leaf", [(1, 2048, 128), (2, 2048, 128), (1, 3001, 256), (2, 3001, 256)])
def test_hss_gemm_vs_dense(P, which, n, leaf):
    A = W.example1(n, which)
    g = np.random.default_rng(which + n)
    m = 777
    X = g.standard_normal((m, n))
    ref = X @ A
    o = P.opts(hss_leaf=leaf, hss_samples=192, hss_samples_inc=64)
    C, rank = P.hss_gemm(_colmajor(A), _colmajor(X), o=o)
    C = C.cpu().numpy()
    err = np.linalg.norm(C - ref) / np.linalg.norm(ref)
    print(f"\n[example1 mat{which} n={n}] rank {rank} relative error {err:.2e}")
    assert rank >= 1
    if which == 1:
        assert rank <= 4  # exact off-diagonal rank 2 (the floor may keep a rounding direction or two)
    assert err <= 1e-12


@pytest.mark.gpu
def test_hss_gemm_dense_fallback(P):
    n, m = 1500, 300
    A = W.example1(n, 2)
    X = np.random.default_rng(3).standard_normal((m, n))
    C, rank = P.hss_gemm(_colmajor(A), _colmajor(X), o=P.opts(force_fail=P.FAIL_HSS))
    assert rank == -1
    ref = X @ A
    assert np.linalg.norm(C.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-14
