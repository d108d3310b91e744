"""Batched solves of uneven sizes: one launch per kernel per tree height across the
batch, the prepare/launch split, and HIP-graph replays (on the GPU).

Graph replays are checked against the eager result each time, with eager work
and synchronisation between replays, and with the inputs changed in place
between replays (a replay must solve the current inputs).
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


def _fill(bs, ds, es):
    bs.d[: sum(bs.sizes)] = torch.tensor(np.concatenate(ds), device=bs.d.device)
    ecat = np.concatenate([x for x in es if x.size] or [np.zeros(0)])
    if ecat.size:
        bs.e[: ecat.size] = torch.tensor(ecat, device=bs.e.device)


def _blocks(bs):
    lam = bs.lam.cpu().numpy()
    Q = bs.Q.cpu().numpy()
    out = []
    for b, n in enumerate(bs.sizes):
        out.append((lam[bs.off[b]:bs.off[b] + n], Q[bs.qoff[b]:bs.qoff[b] + n * n].reshape(n, n).T))
    return out


def test_batched_uneven_sizes_vs_oracle(P, orc):
    sizes = W.batch_sizes(60, 32, 400, seed=3).tolist() + [1, 2, 31, 33, 0]
    ds, es = W.normal_batch(sizes, seed=3)
    lam, Q, off, qoff = P.stedc_batched(sizes, np.concatenate(ds), np.concatenate(es))
    lam, Q = lam.cpu().numpy(), Q.cpu().numpy()
    for b in range(0, len(sizes), 7):
        n = sizes[b]
        if n == 0:
            continue
        lr, _, _ = orc.stedc(ds[b], es[b])
        lb = lam[off[b]:off[b] + n]
        Qb = Q[qoff[b]:qoff[b] + n * n].reshape(n, n).T
        assert np.abs(lb - lr).max() <= 1e-13 * np.abs(lr).max()
        assert orth(Qb) <= 1e-12
        assert residual(ds[b], es[b], lb, Qb) <= 1e-13


def test_batched_equals_single_solves(P):
    sizes = [100, 257, 64, 1000]
    ds, es = W.normal_batch(sizes, seed=4)
    lam, Q, off, qoff = P.stedc_batched(sizes, np.concatenate(ds), np.concatenate(es))
    for b, n in enumerate(sizes):
        l1, Q1 = P.stedc(ds[b], es[b])
        assert torch.equal(l1, lam[off[b]:off[b] + n])
        assert torch.equal(Q1.t().contiguous().reshape(-1), Q[qoff[b]:qoff[b] + n * n])


@pytest.mark.parametrize("mode", ["fp64", "split"])
def test_graph_replay_matches_eager(P, mode):
    sizes = W.batch_sizes(40, 32, 300, seed=5).tolist()
    o = P.opts(gemm_mode=P.GEMM_FP64 if mode == "fp64" else P.GEMM_SPLIT)
    bs = P.BatchedSolver(sizes, o)
    rounds = []
    for r in range(3):
        ds, es = W.normal_batch(sizes, seed=10 + r)
        rounds.append((ds, es))
    # eager reference for each input set
    ref = []
    for ds, es in rounds:
        _fill(bs, ds, es)
        bs.prepare()
        bs.launch()
        torch.cuda.synchronize()
        assert P.status(bs.work) == 0
        ref.append((bs.lam.clone(), bs.Q.clone()))
    _fill(bs, *rounds[0])
    bs.prepare()
    bs.capture()
    for r, (ds, es) in enumerate(rounds * 2):
        _fill(bs, ds, es)
        torch.cuda.synchronize()
        bs.replay()
        # eager work between replays
        x = torch.randn(1000, 1000, device="cuda", dtype=torch.float64)
        (x @ x).sum().item()
        torch.cuda.synchronize()
        assert P.status(bs.work) == 0
        assert torch.equal(bs.lam, ref[r % 3][0]) and torch.equal(bs.Q, ref[r % 3][1]), f"replay {r} differs"
    # and the replays are correct solves
    for b, (lb, Qb) in enumerate(_blocks(bs)[:5]):
        ds, es = rounds[(len(rounds) * 2 - 1) % 3]
        assert orth(Qb) <= (1e-11 if mode == "split" else 1e-12)
        assert residual(ds[b], es[b], lb, Qb) <= (1e-12 if mode == "split" else 1e-13)


def test_batched_full_size_4096(P, orc):
    # The batched workload at its stated size: 4096 tridiagonals, n_b iid U{32..1024}
    # (seed 0), d, e iid N(0,1).  Every matrix: orthogonality and residual of its
    # eigenvectors, computed on the GPU.  64 sampled matrices (the largest among them):
    # eigenvalues against the oracle.  The prepared, graph-replayed launch must give
    # the same bits as the direct call.
    sizes = W.batch_sizes(4096, 32, 1024, seed=0).tolist()
    ds, es = W.normal_batch(sizes, seed=0)
    dcat, ecat = np.concatenate(ds), np.concatenate(es)
    lam, Q, off, qoff = P.stedc_batched(sizes, dcat, ecat)
    dt = torch.tensor(dcat, device="cuda")
    et = torch.tensor(ecat, device="cuda")
    orths, ress = [], []
    eo = 0
    for b, n in enumerate(sizes):
        Qb = Q[qoff[b]:qoff[b] + n * n].view(n, n).t()  # column k = eigenvector k
        lb = lam[off[b]:off[b] + n]
        G = Qb.T @ Qb
        G.diagonal().sub_(1.0)
        orths.append(G.abs().max())
        db, eb = dt[off[b]:off[b] + n], et[eo:eo + n - 1]
        eo += n - 1
        R = db[:, None] * Qb - Qb * lb[None, :]
        R[:-1] += eb[:, None] * Qb[1:]
        R[1:] += eb[:, None] * Qb[:-1]
        ress.append(torch.linalg.norm(R) / (n * lb.abs().max()))
    worst_orth = torch.stack(orths).max().item()
    worst_res = torch.stack(ress).max().item()
    assert worst_orth <= 1e-12, worst_orth
    assert worst_res <= 1e-13, worst_res
    pick = set(np.random.default_rng(0).choice(len(sizes), 63, replace=False).tolist())
    pick.add(int(np.argmax(sizes)))
    lam_h = lam.cpu().numpy()
    for b in sorted(pick):
        n = sizes[b]
        lr, _, _ = orc.stedc(ds[b], es[b])
        assert np.abs(lam_h[off[b]:off[b] + n] - lr).max() <= 1e-13 * np.abs(lr).max(), b
    # the same batch planned once and replayed from a HIP graph: identical bits
    bs = P.BatchedSolver(sizes, P.opts())
    bs.d[: len(dcat)] = dt
    bs.e[: len(ecat)] = torch.tensor(ecat, device="cuda")
    bs.prepare()
    bs.capture()
    for _ in range(2):
        bs.replay()
        torch.cuda.synchronize()
        assert P.status(bs.work) == 0
        assert torch.equal(bs.lam[: len(dcat)], lam) and torch.equal(bs.Q[: Q.numel()], Q)
