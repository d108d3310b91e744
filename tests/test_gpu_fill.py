"""Zero fill of the caller's eigenvector matrix ahead of a root merge (on the GPU).

A root merge of at least 256 rows in the last level of the tree has its output
zero-filled on a second stream while the levels below run (the even depths
below such a root keep their eigenvectors in a workspace buffer of their own;
from 2048 rows the fill comes in two parts: off-diagonal quadrants, then
diagonal halves).  The root then copies only the rows of each deflated column
that can be nonzero.  Here
the caller's buffer starts out as NaN, so an entry that neither the fill nor
the merge writes shows up in every check; deflation is made heavy (tiny
couplings) so that most columns take the short copy.
"""
import ctypes

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


def _deflating(n, seed):
    """d iid U[-1, 1]; every third coupling 1e-18 (type-1 deflation at every
    merge), the others iid U[-1, 1]."""
    d, e = W.uniform(n, seed)
    e = e.copy()
    e[::3] = 1e-18
    return d, e


def _solve_poisoned(P, d, e, o=None):
    lib = P.load()
    o = o or P.opts()
    n = len(d)
    dt = torch.tensor(d, device="cuda")
    et = torch.tensor(e if n > 1 else [0.0], device="cuda")
    lam = torch.empty(n, dtype=torch.float64, device="cuda")
    qbuf = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
    nb = ctypes.c_size_t()
    P._check(lib.phdc_stedc_workspace(n, ctypes.byref(o), ctypes.byref(nb)), "phdc_stedc_workspace")
    work = P.workspace(nb.value, "cuda")
    P._check(lib.phdc_stedc(n, P._ptr(dt), P._ptr(et), P._ptr(lam), P._ptr(qbuf), n, P._ptr(work), work.numel(),
                            ctypes.byref(o), P._stream()), "phdc_stedc")
    assert P.status(work) == 0
    return lam, qbuf.t(), work


def _check_solution(d, e, lam, Q, orc):
    Qh = Q.cpu().numpy()
    lh = lam.cpu().numpy()
    assert np.isfinite(Qh).all(), "entries of Q left unwritten"
    assert orth(Qh) <= 1e-12
    assert residual(d, e, lh, Qh) <= 1e-13
    lr, _, _ = orc.stedc(d, e)
    assert np.abs(lh - lr).max() <= 1e-13 * np.abs(lr).max()


@pytest.mark.parametrize("n", [300, 1000, 2047, 2048, 2500])
def test_single_solve_over_poisoned_q(P, orc, n):
    d, e = _deflating(n, seed=n)
    lam, Q, work = _solve_poisoned(P, d, e)
    tb = P.merge_table(work)
    root = tb[:, 15] > 0
    assert root.sum() == 1 and tb[root, 16][0] == 1
    _check_solution(d, e, lam, Q, orc)
    # the root's copy wrote exactly the rows the fill left to it
    copied = int(P.copied_rows(tb)[root][0])
    ranged = int(P.deflated_rows(tb)[root][0])
    ndefl = int(tb[root, 6][0] + tb[root, 7][0])
    assert ndefl > n // 4
    assert copied == ranged


def test_small_root_takes_no_fill(P, orc):
    d, e = _deflating(255, seed=1)
    lam, Q, work = _solve_poisoned(P, d, e)
    tb = P.merge_table(work)
    assert (tb[:, 16] == 0).all()
    _check_solution(d, e, lam, Q, orc)


@pytest.mark.parametrize("sizes", [[2048, 1900, 1000, 300, 40], [1000, 700, 600, 40, 300, 1]])
def test_batched_over_poisoned_q(P, orc, sizes):
    # Only the roots in the last level (the tallest trees: heights 7 and 6 at
    # leaf size 16) are filled: 2048 (in two parts) and 1900; in the second
    # batch 1000, 700 and 600.
    lib = P.load()
    o = P.opts()
    mats = [_deflating(n, seed=100 + i) for i, n in enumerate(sizes)]
    B = len(sizes)
    off, qoff, acc, qacc = [], [], 0, 0
    for n in sizes:
        off.append(acc)
        qoff.append(qacc)
        acc += n
        qacc += n * n
    arr = lambda v: (ctypes.c_int64 * B)(*v)
    dt = torch.tensor(np.concatenate([m[0] for m in mats]), device="cuda")
    et = torch.tensor(np.concatenate([m[1] for m in mats]), device="cuda")
    lam = torch.empty(acc, dtype=torch.float64, device="cuda")
    Q = torch.full((qacc,), float("nan"), dtype=torch.float64, device="cuda")
    nb = ctypes.c_size_t()
    P._check(lib.phdc_stedc_batched_workspace(B, arr(sizes), ctypes.byref(o), ctypes.byref(nb)), "workspace")
    work = P.workspace(nb.value, "cuda")
    P._check(lib.phdc_stedc_batched(B, arr(sizes), arr(off), arr(qoff), P._ptr(dt), P._ptr(et), P._ptr(lam),
                                    P._ptr(Q), P._ptr(work), work.numel(), ctypes.byref(o), P._stream()),
             "phdc_stedc_batched")
    assert P.status(work) == 0
    tb = P.merge_table(work)
    roots = tb[tb[:, 15] > 0]
    modes = {int(r[0]): int(r[16]) for r in roots}
    for n in sizes:
        if n < 256:
            assert modes.get(n, 0) == 0
    if max(sizes) == 2048:
        assert modes[2048] == 1 and modes[1900] == 1 and modes[1000] == 0 and modes[300] == 0
    else:
        assert modes[1000] == 1 and modes[700] == 1 and modes[600] == 1 and modes[300] == 0
    for b, n in enumerate(sizes):
        Qb = Q[qoff[b]:qoff[b] + n * n].view(n, n).t()
        _check_solution(mats[b][0], mats[b][1], lam[off[b]:off[b] + n], Qb, orc)
    # each matrix's solve equals its single solve, bit for bit
    for b, n in enumerate(sizes):
        l1, Q1 = P.stedc(mats[b][0], mats[b][1])
        assert torch.equal(l1, lam[off[b]:off[b] + n])
        assert torch.equal(Q1.t().contiguous().reshape(-1), Q[qoff[b]:qoff[b] + n * n])
