"""GEMM tile autotuner (on the GPU): the table is filled with measured choices and
the choice changes nothing but speed.

Both tile edges (64 and 128) accumulate every output entry over k in the same
order, so a solve planned before tuning and one planned after are bitwise equal.
The default table already uses both edges (64 up to m = 256, 128 above), so a
solve of n = 2047 runs both kernels.
"""
import numpy as np
import pytest
import torch

import workloads as W
from checks import orth, residual

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1612_07526_amd as P
    P.load()
    return P


def test_autotune_fills_table_and_keeps_results(P):
    d, e = W.toeplitz_121(2047, 1.0)  # no deflation at the top merges: K = m
    l0, Q0 = P.stedc(d, e)
    table = P.autotune_gemm(2048)
    for b in range(6, 12):  # buckets of m = 64 .. 2048
        assert table[b] in (32, 64, 128)
    l1, Q1 = P.stedc(d, e)
    assert torch.equal(l0, l1)
    assert torch.equal(Q0, Q1)
    lam, Q = l1.cpu().numpy(), Q1.cpu().numpy()
    assert orth(Q) <= 1e-12
    assert residual(d, e, lam, Q) <= 1e-13


def test_batched_after_autotune_matches_single(P):
    sizes = [200, 700, 64, 1000]
    ds, es = W.normal_batch(sizes, seed=8)
    lam, Q, off, qoff = P.stedc_batched(sizes, np.concatenate(ds), np.concatenate(es))
    for b, n in enumerate(sizes):
        l1, Q1 = P.stedc(ds[b], es[b])
        assert torch.equal(l1, lam[off[b]:off[b] + n])
        assert torch.equal(Q1.t().contiguous().reshape(-1), Q[qoff[b]:qoff[b] + n * n])
