"""phdc_stedc_noalloc (the solve whose workspace is the library's static device
array) against phdc_stedc (caller-allocated workspace) through the C-ABI: the
same kernels on the same plan, so the results must be bitwise equal.  Two calls
in a row, the second with a smaller input, to check that the shared array is
re-planned and re-cleared; an input too large for the array and the HSS form
are refused with their documented codes."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1612_07526_amd as P
    P.load()
    return P


def _noalloc(P, d, e, o):
    lib = P.load()
    n = len(d)
    dt = torch.tensor(d, device="cuda")
    et = torch.tensor(e if len(e) else np.zeros(1), device="cuda")
    lam = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    Q = torch.full((n, n), np.nan, dtype=torch.float64, device="cuda")
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    rc = lib.phdc_stedc_noalloc(n, P._ptr(dt), P._ptr(et), P._ptr(lam), P._ptr(Q), n, P._ptr(info), ctypes.byref(o),
                                P._stream())
    torch.cuda.synchronize()
    return rc, int(info.item()), lam, Q.t()


@pytest.mark.parametrize("mode", ["fp64", "split"])
def test_noalloc_matches_stedc(P, mode):
    gm = P.GEMM_FP64 if mode == "fp64" else P.GEMM_SPLIT
    cases = [(2400, 1, 16), (777, 2, 32)] if mode == "fp64" else [(1500, 3, 32), (300, 4, 16)]
    for n, seed, leaf in cases:  # second call smaller than the first
        d, e = W.uniform(n, seed)
        o = P.opts(leaf_size=leaf, gemm_mode=gm)
        rc, info, lam, Q = _noalloc(P, d, e, o)
        assert rc == 0 and info == 0, (rc, info)
        lam_ref, Q_ref = P.stedc(d, e, o=o)
        assert torch.equal(lam, lam_ref), n
        assert torch.equal(Q, Q_ref), n


def test_noalloc_refusals(P):
    lib = P.load()
    o = P.opts()
    v = ctypes.c_void_p
    fake = v(0x1000)  # never dereferenced: every call below fails its host-side checks first
    nb = ctypes.c_size_t()
    n_big = 4096
    assert lib.phdc_stedc_workspace(n_big, ctypes.byref(o), ctypes.byref(nb)) == 0
    assert nb.value > P.NOALLOC_SCRATCH_BYTES
    assert lib.phdc_stedc_noalloc(n_big, fake, fake, fake, fake, n_big, fake, ctypes.byref(o), v(0)) == -1
    assert lib.phdc_stedc_noalloc(100, fake, fake, fake, fake, 100, v(0), ctypes.byref(o), v(0)) == -7
    oh = P.opts(gemm_mode=P.GEMM_HSS)
    assert lib.phdc_stedc_noalloc(100, fake, fake, fake, fake, 100, fake, ctypes.byref(oh), v(0)) == -8
    # a status from the device comes back through info
    d, e = W.uniform(500, 5)
    rc, info, _, _ = _noalloc(P, d, e, P.opts(force_fail=P.FAIL_SECULAR))
    assert rc == 0 and info == P.STATUS_SECULAR
