"""The boundary's error contract (on the GPU), through the C-ABI.

* One test per device status code: PHDC_ERR_LEAF and PHDC_ERR_SECULAR through the
  force_fail test hooks (the bounded QL / secular loops get no iterations, so every
  kernel still exits normally), PHDC_ERR_UNSORTED (unsorted merge poles) and
  PHDC_ERR_NONFINITE (a NaN in z; a NaN in the poles).
* opts.check_finite: the device scan makes the entry point return -(index of the
  offending array argument) and sets PHDC_ERR_NONFINITE, for stedc, merge and the
  batched solve; the prepared (graph) launch only sets the status.
* The HSS fall-back (Sec. 2.2: Gu's FP64 products whenever HSS does not apply):
  with the PHDC_FAIL_HSS hook every compression gives up, and the merge must still
  meet the FP64 bounds, reporting path 0 and HSS rank -1.
* A prepared plan is forgotten by any later solve on the same workspace and by
  phdc_release: phdc_launch_prepared then returns -1 instead of launching stale grids.
"""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from checks import orth, residual, vector_error_ratio

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1612_07526_amd as P
    P.load()
    return P


def _np(t):
    return t.detach().cpu().numpy()


def _raw_stedc(P, d, e, o):
    """phdc_stedc through the C-ABI: returns (return code, device status, lam, Q)."""
    lib = P.load()
    n = len(d)
    dt = torch.tensor(d, device="cuda")
    et = torch.tensor(e if len(e) else np.zeros(1), device="cuda")
    lam = torch.empty(n, dtype=torch.float64, device="cuda")
    Q = torch.empty((n, n), dtype=torch.float64, device="cuda")
    nb = ctypes.c_size_t()
    assert lib.phdc_stedc_workspace(n, ctypes.byref(o), ctypes.byref(nb)) == 0
    work = P.workspace(nb.value, "cuda")
    rc = lib.phdc_stedc(n, P._ptr(dt), P._ptr(et), P._ptr(lam), P._ptr(Q), n, P._ptr(work), work.numel(),
                        ctypes.byref(o), P._stream())
    st = P.status(work)
    P.release(work)
    return rc, st, lam, Q


def test_status_leaf_forced(P):
    d, e = W.uniform(200, 3)
    rc, st, lam, Q = _raw_stedc(P, d, e, P.opts(force_fail=P.FAIL_LEAF))
    assert rc == 0 and st == P.STATUS_LEAF
    # the same solve without the hook is clean
    rc, st, lam, Q = _raw_stedc(P, d, e, P.opts())
    assert rc == 0 and st == P.STATUS_OK


def test_status_secular_forced(P):
    d, e = W.uniform(200, 3)
    rc, st, _, _ = _raw_stedc(P, d, e, P.opts(force_fail=P.FAIL_SECULAR))
    assert rc == 0 and st == P.STATUS_SECULAR
    D, z, rho, Q1, Q2 = W.random_merge(30, 40, seed=2)
    _, _, work = P.merge(D, z, rho, torch.tensor(Q1), torch.tensor(Q2), o=P.opts(force_fail=P.FAIL_SECULAR),
                         check=False, return_work=True)
    assert P.status(work) == P.STATUS_SECULAR


def test_status_unsorted(P):
    g = np.random.default_rng(1)
    D = g.standard_normal(20)
    _, _, work = P.merge(D, g.standard_normal(20), 1.0, torch.tensor(W.random_orthogonal(10, g)),
                         torch.tensor(W.random_orthogonal(10, g)), check=False, return_work=True)
    assert P.status(work) == P.STATUS_UNSORTED


def test_status_nonfinite_in_z(P):
    # a NaN in z: nothing may pass for converged (the secular function is NaN)
    D, z, rho, Q1, Q2 = W.random_merge(50, 60, seed=4)
    z[17] = np.nan
    _, _, work = P.merge(D, z, rho, torch.tensor(Q1), torch.tensor(Q2), check=False, return_work=True)
    assert P.status(work) == P.STATUS_NONFINITE


def test_status_nonfinite_in_poles(P):
    D, z, rho, Q1, Q2 = W.random_merge(50, 60, seed=5)
    D[70] = np.inf
    _, _, work = P.merge(D, z, rho, torch.tensor(Q1), torch.tensor(Q2), check=False, return_work=True)
    assert P.status(work) == P.STATUS_NONFINITE


@pytest.mark.parametrize("case", ["ok", "unsorted", "nan_z", "inf_d"])
def test_status_large_merge(P, case):
    # merges of 4096 rows and more deflate across many workgroups; bad input is
    # handed back to the one-workgroup path, which reports it
    D, z, rho, Q1, Q2 = W.random_merge(2048, 2048, seed=11)
    if case == "unsorted":
        D[100], D[101] = D[101], D[100] + 1.0
    elif case == "nan_z":
        z[3000] = np.nan
    elif case == "inf_d":
        D[2500] = np.inf
    lam, Q, work = P.merge(D, z, rho, torch.tensor(Q1), torch.tensor(Q2), check=False, return_work=True)
    st = P.status(work)
    if case == "ok":
        # each eigenvalue sits where the secular function counts it (a Sturm-type
        # count over the poles, as in the full-size merge test); orthogonality
        assert st == P.STATUS_OK
        lh = _np(lam)
        order = np.argsort(D, kind="stable")
        ds, zs = D[order], z[order] / np.linalg.norm(z)
        r = rho * float(np.dot(z, z))
        delta = 1e-13 * np.abs(lh).max()

        def below(x):
            j = int(np.searchsorted(ds, x, side="left"))
            return 0 if j == 0 else j - 1 + (1 if 1.0 + r * np.sum(zs * zs / (ds - x)) > 0 else 0)

        for k in np.random.default_rng(2).choice(D.size, 32, replace=False):
            assert below(lh[k] - delta) <= k and below(lh[k] + delta) >= k + 1
        assert orth(_np(Q)) <= 1e-12
    else:
        assert st == (P.STATUS_UNSORTED if case == "unsorted" else P.STATUS_NONFINITE)


def test_status_nonfinite_in_stedc_input(P):
    # without the scan a NaN in d is caught by the first kernel that meets it
    d, e = W.uniform(300, 6)
    d[123] = np.nan
    rc, st, _, _ = _raw_stedc(P, d, e, P.opts())
    assert rc == 0 and st in (P.STATUS_LEAF, P.STATUS_NONFINITE)


@pytest.mark.parametrize("where,expect", [("d", -2), ("e", -3), ("none", 0)])
def test_check_finite_stedc(P, where, expect):
    d, e = W.uniform(257, 7)
    if where == "d":
        d[5] = np.inf
    if where == "e":
        e[200] = np.nan
    rc, st, lam, Q = _raw_stedc(P, d, e, P.opts(check_finite=1))
    assert rc == expect
    assert st == (P.STATUS_OK if expect == 0 else P.STATUS_NONFINITE)
    if expect == 0:
        assert orth(_np(Q).T) <= 1e-12


@pytest.mark.parametrize("where,expect", [("D", -3), ("z", -4)])
def test_check_finite_merge(P, where, expect):
    lib = P.load()
    D, z, rho, Q1, Q2 = W.random_merge(20, 30, seed=8)
    if where == "D":
        D[3] = np.nan
    else:
        z[40] = np.inf
    o = P.opts(check_finite=1)
    m = 50
    Dt, zt = torch.tensor(D, device="cuda"), torch.tensor(z, device="cuda")
    Q1c, ld1 = P._colmajor(torch.tensor(Q1, device="cuda"))
    Q2c, ld2 = P._colmajor(torch.tensor(Q2, device="cuda"))
    lam = torch.empty(m, dtype=torch.float64, device="cuda")
    Q = torch.empty((m, m), dtype=torch.float64, device="cuda")
    nb = ctypes.c_size_t()
    assert lib.phdc_merge_workspace(20, 30, ctypes.byref(o), ctypes.byref(nb)) == 0
    work = P.workspace(nb.value, "cuda")
    rc = lib.phdc_merge(20, 30, P._ptr(Dt), P._ptr(zt), rho, P._ptr(Q1c), ld1, P._ptr(Q2c), ld2, P._ptr(lam),
                        P._ptr(Q), m, P._ptr(work), work.numel(), ctypes.byref(o), P._stream())
    assert rc == expect
    assert P.status(work) == P.STATUS_NONFINITE


def test_check_finite_batched_and_prepared(P):
    sizes = [40, 70, 33]
    ds, es = W.normal_batch(sizes, seed=9)
    es[1][10] = np.nan
    with pytest.raises(P.PhdcError, match="returned -6"):
        P.stedc_batched(sizes, np.concatenate(ds), np.concatenate(es), o=P.opts(check_finite=1))
    # the prepared launch (capturable: no waiting) only sets the status word
    bs = P.BatchedSolver(sizes, P.opts(check_finite=1))
    bs.d[: sum(sizes)] = torch.tensor(np.concatenate(ds), device="cuda")
    ecat = np.concatenate(es)
    bs.e[: ecat.size] = torch.tensor(ecat, device="cuda")
    bs.prepare()
    bs.launch()
    assert P.status(bs.work) == P.STATUS_NONFINITE
    ecat[~np.isfinite(ecat)] = 0.5
    bs.e[: ecat.size] = torch.tensor(ecat, device="cuda")
    bs.launch()
    assert P.status(bs.work) == P.STATUS_OK


@pytest.mark.parametrize("N", [600, 2048])
def test_hss_fallback_merge(P, orc, N):
    D, z, rho, Q1, Q2 = W.fig3_merge(N, seed=2)
    o = P.opts(gemm_mode=P.GEMM_HSS, hss_min_K=256, hss_leaf=128, hss_samples=192, hss_samples_inc=64,
               force_fail=P.FAIL_HSS)
    lref, Qref, _ = orc.merge(D, z, rho, Q1, Q2)
    lam, Q, work = P.merge(D, z, rho, torch.tensor(Q1), torch.tensor(Q2), o=o, return_work=True)
    st = P.merge_stats(work)
    assert st[0] == N and st[6] == 0 and st[7] == -1  # FP64 product, compression abandoned
    lam, Q = _np(lam), _np(Q)
    assert np.abs(lam - lref).max() <= 1e-13 * np.abs(lref).max()
    assert orth(Q) <= 1e-12
    ratio, ncols = vector_error_ratio(Q, Qref, lref)
    assert ratio <= 1.0, ratio


def test_hss_fallback_stedc(P):
    # Toeplitz n = 2047: the top merges keep every pole, the compression is abandoned at
    # each of them and the FP64 product finishes the solve
    n = 2047
    d, e = W.toeplitz_121(n, 1.0)
    o = P.opts(gemm_mode=P.GEMM_HSS, hss_min_K=512, hss_leaf=128, hss_samples=192, force_fail=P.FAIL_HSS)
    lam, Q, work = P.stedc(d, e, o=o, return_work=True)
    tab = P.merge_table(work)
    big = tab[:, 2] >= 512
    assert big.any() and np.all(tab[big, 8] == 0) and np.all(tab[big, 9] == -1)
    lam, Q = _np(lam), _np(Q)
    k = np.arange(1, n + 1)
    assert np.abs(lam - np.sort(2.0 + 2.0 * np.cos(k * np.pi / (n + 1)))).max() <= 4e-13
    assert orth(Q) <= 1e-12 and residual(d, e, lam, Q) <= 1e-13


def test_prepared_plan_is_forgotten(P):
    sizes = [50, 90]
    ds, es = W.normal_batch(sizes, seed=11)
    bs = P.BatchedSolver(sizes, P.opts())
    bs.d[: sum(sizes)] = torch.tensor(np.concatenate(ds), device="cuda")
    ecat = np.concatenate(es)
    bs.e[: ecat.size] = torch.tensor(ecat, device="cuda")
    bs.prepare()
    lib = P.load()
    assert lib.phdc_launch_prepared(P._ptr(bs.work), P._stream()) == 0
    # another solve on the same workspace replaces the plan on the device
    P.stedc_batched([30], np.ones(30), np.ones(29), work=bs.work)
    assert lib.phdc_launch_prepared(P._ptr(bs.work), P._stream()) == -1
    bs.prepare()
    assert lib.phdc_launch_prepared(P._ptr(bs.work), P._stream()) == 0
    assert P.status(bs.work) == 0
    P.release(bs.work)
    assert lib.phdc_launch_prepared(P._ptr(bs.work), P._stream()) == -1
    assert lib.phdc_release(None) == -1
