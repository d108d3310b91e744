"""MI355X (gfx950) divide-and-conquer tridiagonal eigensolver.

Thin Python binding of ``libphdc.so`` (C-ABI declared in ``include/phdc.h``).
This module only marshals arguments: every step of the solve runs in the HIP
kernels of the library.  Device memory and streams come from PyTorch.  If the
library is missing, every entry point raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphdc.so")

GEMM_FP64 = 0
GEMM_SPLIT = 1
GEMM_HSS = 2

STATUS_OK, STATUS_LEAF, STATUS_SECULAR, STATUS_UNSORTED, STATUS_NONFINITE = 0, 1, 2, 3, 4
STATUS_TEXT = {0: "ok", 1: "leaf QL did not converge", 2: "secular root did not converge",
               3: "merge input D1/D2 not ascending", 4: "non-finite input"}
E_HIP = -100  # host-side return code: a HIP runtime call failed
NOALLOC_SCRATCH_BYTES = 96 << 20  # static workspace of phdc_stedc_noalloc (PHDC_NOALLOC_SCRATCH_BYTES)
# bits of Opts.force_fail (test hooks)
FAIL_LEAF, FAIL_SECULAR, FAIL_HSS = 1, 2, 4


class Opts(ctypes.Structure):
    _fields_ = [
        ("leaf_size", ctypes.c_int32),
        ("gemm_mode", ctypes.c_int32),
        ("hss_min_K", ctypes.c_int64),
        ("hss_rel_tol", ctypes.c_double),
        ("hss_leaf", ctypes.c_int32),
        ("hss_samples", ctypes.c_int32),
        ("hss_samples_inc", ctypes.c_int32),
        ("split_slices", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("canonical_sign", ctypes.c_int32),
        ("check_finite", ctypes.c_int32),
        ("force_fail", ctypes.c_int32),
    ]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t


class PhdcError(RuntimeError):
    pass


def load():
    """Load libphdc.so (built by ``build.py``); raise if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise PhdcError(f"{LIB_PATH} is missing: build it with `python -m paper_1612_07526_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.phdc_opts_default.argtypes = [P(Opts)]
    lib.phdc_opts_default.restype = None
    lib.phdc_version.restype = ctypes.c_int
    lib.phdc_stedc_workspace.argtypes = [_i64, P(Opts), P(_sz)]
    lib.phdc_stedc.argtypes = [_i64, _vp, _vp, _vp, _vp, _i64, _vp, _sz, P(Opts), _vp]
    lib.phdc_merge_workspace.argtypes = [_i64, _i64, P(Opts), P(_sz)]
    lib.phdc_merge.argtypes = [_i64, _i64, _vp, _vp, ctypes.c_double, _vp, _i64, _vp, _i64, _vp, _vp, _i64,
                               _vp, _sz, P(Opts), _vp]
    lib.phdc_stedc_batched_workspace.argtypes = [_i64, P(_i64), P(Opts), P(_sz)]
    lib.phdc_stedc_batched.argtypes = [_i64, P(_i64), P(_i64), P(_i64), _vp, _vp, _vp, _vp, _vp, _sz, P(Opts),
                                       _vp]
    lib.phdc_secular.argtypes = [_i64, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _sz, _vp]
    lib.phdc_status.argtypes = [_vp, _vp]
    lib.phdc_release.argtypes = [_vp]
    lib.phdc_merge_stats.argtypes = [_vp, P(ctypes.c_int32)]
    lib.phdc_stedc_batched_prepare.argtypes = [_i64, P(_i64), P(_i64), P(_i64), _vp, _vp, _vp, _vp, _vp, _sz,
                                               P(Opts), _vp]
    lib.phdc_launch_prepared.argtypes = [_vp, _vp]
    lib.phdc_stedc_backward_workspace.argtypes = [_i64, _i64, P(_sz)]
    lib.phdc_stedc_backward.argtypes = [_i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
    lib.phdc_merge_table.argtypes = [_vp, _i64, P(ctypes.c_int32), P(_i64)]
    lib.phdc_profile_enable.argtypes = [ctypes.c_int]
    lib.phdc_profile_read.argtypes = [P(ctypes.c_double), P(_i64), ctypes.c_int]
    lib.phdc_profile_select.argtypes = [ctypes.c_uint32]
    lib.phdc_autotune_gemm_workspace.argtypes = [_i64, P(_sz)]
    lib.phdc_autotune_gemm.argtypes = [_i64, _vp, _sz, _vp]
    lib.phdc_gemm_tile_table.argtypes = [P(ctypes.c_int32), ctypes.c_int]
    lib.phdc_stedc_noalloc.argtypes = [_i64, _vp, _vp, _vp, _vp, _i64, _vp, P(Opts), _vp]
    lib.phdc_hss_gemm_workspace.argtypes = [_i64, _i64, P(Opts), P(_sz)]
    lib.phdc_hss_gemm.argtypes = [_i64, _vp, _i64, _i64, _vp, _i64, _vp, _i64, P(ctypes.c_int32), _vp, _sz, P(Opts),
                                  _vp]
    _lib = lib
    return lib


EXPORTS = ["phdc_stedc_batched_prepare", "phdc_launch_prepared", "phdc_opts_default", "phdc_version", "phdc_stedc_workspace", "phdc_stedc", "phdc_merge_workspace",
           "phdc_merge", "phdc_stedc_batched_workspace", "phdc_stedc_batched", "phdc_stedc_backward_workspace",
           "phdc_stedc_backward", "phdc_status", "phdc_release", "phdc_merge_stats", "phdc_secular", "phdc_merge_table",
           "phdc_profile_enable", "phdc_profile_read", "phdc_profile_select", "phdc_autotune_gemm_workspace",
           "phdc_autotune_gemm",
           "phdc_gemm_tile_table", "phdc_hss_gemm_workspace", "phdc_hss_gemm", "phdc_stedc_noalloc"]


def autotune_gemm(max_m: int = 4096, device="cuda", stream=None) -> list:
    """Time the FP64 update-GEMM tile rules (32-, 64- and 128-wide tiles) on synthetic merges
    of size 64..max_m and record the fastest per size bucket (used by every solve planned
    afterwards).
    Returns the tile table (entry b: bucket 2^(b-1) < m <= 2^b; 0 = not timed)."""
    lib = load()
    nb = _sz()
    _check(lib.phdc_autotune_gemm_workspace(int(max_m), ctypes.byref(nb)), "phdc_autotune_gemm_workspace")
    work = workspace(nb.value, device)
    _check(lib.phdc_autotune_gemm(int(max_m), _ptr(work), nb.value, _stream(stream)), "phdc_autotune_gemm")
    return gemm_tile_table()


def gemm_tile_table() -> list:
    buf = (ctypes.c_int32 * 32)()
    n = load().phdc_gemm_tile_table(buf, 32)
    return list(buf)[:max(n, 0)]

PHASES = ["leaf", "deflate", "rotate", "secular", "loewner", "uhat_norm", "uhat_write", "rank", "gemm", "copy",
          "sign", "split_slice", "split_gemm", "hss_sample", "hss_compress", "hss_apply", "adj_gemm", "adj_band",
          "small_merge", "fill"]


def profile_phases(fn, reps: int = 1, phases=None) -> dict:
    """Run fn() reps times with the library's per-phase HIP-event timing on (all phases,
    or only those named in ``phases``); returns {phase: (ms per rep, launches per rep)}
    for the phases that ran."""
    lib = load()
    torch.cuda.synchronize()
    n = len(PHASES)
    lib.phdc_profile_read((ctypes.c_double * n)(), (_i64 * n)(), n)  # drop anything pending
    mask = 0xFFFFFFFF if phases is None else sum(1 << PHASES.index(p) for p in phases)
    lib.phdc_profile_select(mask)
    lib.phdc_profile_enable(1)
    try:
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
    finally:
        lib.phdc_profile_enable(0)
        lib.phdc_profile_select(0xFFFFFFFF)
    ms = (ctypes.c_double * n)()
    cnt = (_i64 * n)()
    _check(lib.phdc_profile_read(ms, cnt, n), "phdc_profile_read")
    return {PHASES[i]: (ms[i] / reps, cnt[i] // reps) for i in range(n) if cnt[i]}


def opts(**kw) -> Opts:
    o = Opts()
    load().phdc_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() > 0 else 0)


def _check(rc: int, what: str):
    if rc != 0:
        raise PhdcError(f"{what} returned {rc}")


def _dev_f64(x, device) -> torch.Tensor:
    t = torch.as_tensor(x, dtype=torch.float64, device=device)
    return t.contiguous()


def workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def status(work: torch.Tensor, stream=None) -> int:
    return load().phdc_status(_ptr(work), _stream(stream))


def release(work: torch.Tensor) -> None:
    """Drop the library's host-side state for this workspace (call before freeing it)."""
    _check(load().phdc_release(_ptr(work)), "phdc_release")


def merge_stats(work: torch.Tensor) -> list:
    buf = (ctypes.c_int32 * 8)()
    _check(load().phdc_merge_stats(_ptr(work), buf), "phdc_merge_stats")
    return list(buf)


MERGE_TABLE_COLS = 19


def merge_table(work: torch.Tensor):
    """Per-merge sizes of the last solve on `work` as an (nmerges, 19) int32 numpy array:
    m, n1, K, k1, k2, k3, type-1 deflations, type-2 deflations, path (0 FP64, 1 split,
    2 HSS), HSS rank, deflated columns nonzero in the Q1 rows only / both halves / the
    Q2 rows only, rows the deflated columns can be nonzero in (summed; low 32 bits as
    unsigned, then the high bits: see deflated_rows), 1 for the last merge of its matrix,
    1 for a last merge whose output was zero-filled beforehand, and for
    such a merge the rows its deflated-column copy writes (summed, low / high bits: see
    copied_rows).  Rows follow the planning order (the root merge last)."""
    import numpy as np
    lib = load()
    rows = ctypes.c_int64()
    _check(lib.phdc_merge_table(_ptr(work), 0, None, ctypes.byref(rows)), "phdc_merge_table")
    n = rows.value
    buf = (ctypes.c_int32 * max(n * MERGE_TABLE_COLS, 1))()
    _check(lib.phdc_merge_table(_ptr(work), n, buf, ctypes.byref(rows)), "phdc_merge_table")
    return np.frombuffer(buf, dtype=np.int32)[: n * MERGE_TABLE_COLS].reshape(n, MERGE_TABLE_COLS).copy()


def copied_rows(table):
    """Rows the deflated-column copy of each prefilled last merge writes, summed (int64
    numpy array; 0 for other merges), from the two 32-bit columns of merge_table."""
    import numpy as np
    lo = table[:, 17].astype(np.int64) & 0xFFFFFFFF
    return lo + (table[:, 18].astype(np.int64) << 32)


def deflated_rows(table):
    """Rows the deflated columns of each merge can be nonzero in, summed (int64 numpy
    array), from the two 32-bit columns of merge_table."""
    import numpy as np
    lo = table[:, 13].astype(np.int64) & 0xFFFFFFFF
    return lo + (table[:, 14].astype(np.int64) << 32)


def _raise_status(work, stream=None):
    st = status(work, stream)
    if st != 0:
        raise PhdcError(f"device status {st}: {STATUS_TEXT.get(st, '?')}")


def stedc(d, e, o: Opts | None = None, device="cuda", stream=None, work=None, check=True, return_work=False):
    """Eigen-decomposition of the tridiagonal (d, e): returns (lambda ascending, Q) on the GPU.

    Q is returned as an (n, n) column-major view (strides (1, n)); column j is the
    eigenvector of lambda[j].
    """
    lib = load()
    o = o or opts()
    d = _dev_f64(d, device)
    n = d.numel()
    e = _dev_f64(e, d.device) if n > 1 else torch.zeros(1, dtype=torch.float64, device=d.device)
    lam = torch.empty(n, dtype=torch.float64, device=d.device)
    qbuf = torch.empty((n, n), dtype=torch.float64, device=d.device)
    nb = ctypes.c_size_t()
    _check(lib.phdc_stedc_workspace(n, ctypes.byref(o), ctypes.byref(nb)), "phdc_stedc_workspace")
    if work is None or work.numel() < nb.value:
        work = workspace(nb.value, d.device)
    _check(lib.phdc_stedc(n, _ptr(d), _ptr(e), _ptr(lam), _ptr(qbuf), max(n, 1), _ptr(work), work.numel(),
                          ctypes.byref(o), _stream(stream)), "phdc_stedc")
    if check:
        _raise_status(work, stream)
    Q = qbuf.t()
    return (lam, Q, work) if return_work else (lam, Q)


def _colmajor(A: torch.Tensor):
    """Column-major copy of a 2-D tensor: returns (storage tensor, ld)."""
    A = A.to(torch.float64)
    n = A.shape[0]
    return A.t().contiguous(), max(n, 1)


def merge(D, z, rho, Q1, Q2, o: Opts | None = None, device="cuda", stream=None, check=True, return_work=False):
    """One rank-one merge (Eq. (3)-(6)): eigenpairs of diag(Q1,Q2)(D + rho z z^T)diag(Q1,Q2)^T."""
    lib = load()
    o = o or opts()
    D = _dev_f64(D, device)
    z = _dev_f64(z, D.device)
    Q1 = torch.as_tensor(Q1, dtype=torch.float64, device=D.device)
    Q2 = torch.as_tensor(Q2, dtype=torch.float64, device=D.device)
    n1, n2 = Q1.shape[0], Q2.shape[0]
    m = n1 + n2
    Q1c, ld1 = _colmajor(Q1)
    Q2c, ld2 = _colmajor(Q2)
    lam = torch.empty(m, dtype=torch.float64, device=D.device)
    qbuf = torch.empty((m, m), dtype=torch.float64, device=D.device)
    nb = ctypes.c_size_t()
    _check(lib.phdc_merge_workspace(n1, n2, ctypes.byref(o), ctypes.byref(nb)), "phdc_merge_workspace")
    work = workspace(nb.value, D.device)
    _check(lib.phdc_merge(n1, n2, _ptr(D), _ptr(z), float(rho), _ptr(Q1c), ld1, _ptr(Q2c), ld2, _ptr(lam),
                          _ptr(qbuf), max(m, 1), _ptr(work), work.numel(), ctypes.byref(o), _stream(stream)),
           "phdc_merge")
    if check:
        _raise_status(work, stream)
    Q = qbuf.t()
    return (lam, Q, work) if return_work else (lam, Q)


def stedc_batched(sizes, d, e, o: Opts | None = None, device="cuda", stream=None, check=True, work=None,
                  return_work=False):
    """Batched solve.  d: packed diagonals (sum n_b); e: packed off-diagonals (sum (n_b - 1)).

    Returns (lambda packed, Q packed) where matrix b's eigenvectors are the n_b x n_b
    column-major block at Q[qoff_b : qoff_b + n_b^2].
    """
    lib = load()
    o = o or opts()
    sizes = [int(x) for x in sizes]
    B = len(sizes)
    n_arr = (ctypes.c_int64 * max(B, 1))(*sizes)
    off, qoff, acc, qacc = [], [], 0, 0
    for nb_ in sizes:
        off.append(acc)
        qoff.append(qacc)
        acc += nb_
        qacc += nb_ * nb_
    off_arr = (ctypes.c_int64 * max(B, 1))(*off)
    qoff_arr = (ctypes.c_int64 * max(B, 1))(*qoff)
    d = _dev_f64(d, device)
    e = _dev_f64(e, d.device) if e is not None and len(e) else torch.zeros(1, dtype=torch.float64, device=d.device)
    lam = torch.empty(max(acc, 1), dtype=torch.float64, device=d.device)
    Q = torch.empty(max(qacc, 1), dtype=torch.float64, device=d.device)
    nb = ctypes.c_size_t()
    _check(lib.phdc_stedc_batched_workspace(B, n_arr, ctypes.byref(o), ctypes.byref(nb)),
           "phdc_stedc_batched_workspace")
    if work is None or work.numel() < nb.value:
        work = workspace(nb.value, d.device)
    _check(lib.phdc_stedc_batched(B, n_arr, off_arr, qoff_arr, _ptr(d), _ptr(e), _ptr(lam), _ptr(Q), _ptr(work),
                                  work.numel(), ctypes.byref(o), _stream(stream)), "phdc_stedc_batched")
    if check:
        _raise_status(work, stream)
    out = (lam[:acc], Q[:qacc], off, qoff)
    return out + (work,) if return_work else out


def hss_gemm(A: torch.Tensor, X: torch.Tensor, o: Opts | None = None, stream=None, work=None):
    """C = X A with the K x K matrix A compressed to HSS form (Algorithm 1), as in the
    paper's Example 1.  A (K x K) and X (m x K) are float64 CUDA tensors in column-major
    storage: pass them as transposed views of contiguous tensors (``A = At.t()``), or any
    tensor with stride (1, ld).  Returns (C as an (m, K) column-major view, largest ID
    rank or -1 if the dense product was used)."""
    lib = load()
    o = o or opts()
    K, m = A.shape[0], X.shape[0]
    assert A.shape == (K, K) and X.shape[1] == K and A.stride(0) == 1 and X.stride(0) == 1
    Cs = torch.empty((K, m), dtype=torch.float64, device=A.device)
    nb = ctypes.c_size_t()
    _check(lib.phdc_hss_gemm_workspace(K, m, ctypes.byref(o), ctypes.byref(nb)), "phdc_hss_gemm_workspace")
    if work is None or work.numel() < nb.value:
        work = workspace(nb.value, A.device)
    rank = ctypes.c_int32(0)
    _check(lib.phdc_hss_gemm(K, _ptr(A), A.stride(1), m, _ptr(X), X.stride(1), _ptr(Cs), m, ctypes.byref(rank),
                             _ptr(work), work.numel(), ctypes.byref(o), _stream(stream)), "phdc_hss_gemm")
    return Cs.t(), rank.value


def secular(d, z, rho, device="cuda", stream=None, check=True, return_iters=False):
    """Roots of 1 + rho sum z_i^2/(d_i - lambda) as (origin index int32, offset) device tensors
    (and, with return_iters, the largest number of secular-function evaluations of one root)."""
    lib = load()
    d = _dev_f64(d, device)
    z = _dev_f64(z, d.device)
    K = d.numel()
    org = torch.empty(max(K, 1), dtype=torch.int32, device=d.device)
    tau = torch.empty(max(K, 1), dtype=torch.float64, device=d.device)
    work = workspace(256, d.device)
    _check(lib.phdc_secular(K, _ptr(d), _ptr(z), float(rho), _ptr(org), _ptr(tau), _ptr(work), work.numel(),
                            _stream(stream)), "phdc_secular")
    if check:
        _raise_status(work, stream)
    if return_iters:
        return org[:K], tau[:K], int(work[4:8].view(torch.int32).item())
    return org[:K], tau[:K]


def stedc_backward(lam, Qstore, lam_bar, Qbar_store, n: int, batch: int, stream=None):
    """Gradients (d_bar, e_bar) of a loss from (lam_bar, Q_bar) at eigenpairs (lam, Q).

    ``Qstore``/``Qbar_store`` hold `batch` column-major n x n blocks back to back
    (ld = n); ``lam``/``lam_bar`` are packed (batch * n).  ``Qbar_store`` may be None.
    """
    lib = load()
    dev = lam.device
    dbar = torch.empty(max(batch * n, 1), dtype=torch.float64, device=dev)
    ebar = torch.empty(max(batch * (n - 1), 1), dtype=torch.float64, device=dev)
    nb = ctypes.c_size_t()
    _check(lib.phdc_stedc_backward_workspace(n, batch, ctypes.byref(nb)), "phdc_stedc_backward_workspace")
    work = workspace(nb.value, dev)
    _check(lib.phdc_stedc_backward(n, batch, _ptr(lam), _ptr(Qstore), _ptr(lam_bar), _ptr(Qbar_store),
                                   _ptr(dbar), _ptr(ebar), _ptr(work), work.numel(), _stream(stream)),
           "phdc_stedc_backward")
    return dbar[: batch * n].view(batch, n), ebar[: batch * max(n - 1, 0)].view(batch, max(n - 1, 0))


class _TridiagonalEigh(torch.autograd.Function):
    """(d, e) -> (lambda, Q) with eigenvector signs fixed (largest-magnitude entry positive)."""

    @staticmethod
    def forward(ctx, d, e, leaf_size, gemm_mode):
        squeeze = d.dim() == 1
        d2 = d.reshape(1, -1) if squeeze else d
        e2 = e.reshape(1, -1) if squeeze else e
        B, n = d2.shape
        o = opts(canonical_sign=1, leaf_size=leaf_size, gemm_mode=gemm_mode)
        lam, Qp, _, _ = stedc_batched([n] * B, d2.reshape(-1), e2.reshape(-1), o=o, device=d.device)
        lam = lam.view(B, n)
        Qstore = Qp.view(B, n, n)          # Qstore[b, j, i] = Q_b(i, j)
        ctx.save_for_backward(lam, Qstore)
        ctx.squeeze = squeeze
        Q = Qstore.transpose(1, 2)
        if squeeze:
            return lam[0], Q[0]
        return lam, Q

    @staticmethod
    def backward(ctx, glam, gQ):
        lam, Qstore = ctx.saved_tensors
        B, n = lam.shape
        if glam is not None:
            glam = glam.reshape(B, n).to(torch.float64).contiguous()
        gq_store = None
        if gQ is not None:
            gq_store = gQ.reshape(B, n, n).transpose(1, 2).to(torch.float64).contiguous()
        dbar, ebar = stedc_backward(lam, Qstore, glam, gq_store, n, B)
        if ctx.squeeze:
            return dbar[0], ebar[0], None, None
        return dbar, ebar, None, None


def eigh_tridiagonal(d: torch.Tensor, e: torch.Tensor, leaf_size: int = 32, gemm_mode: int = GEMM_FP64):
    """Differentiable eigen-decomposition of symmetric tridiagonal matrices on the GPU.

    d: (n,) or (B, n) float64 CUDA tensor; e: (n-1,) or (B, n-1).  Returns (lambda, Q)
    with lambda ascending and Q[..., :, j] the eigenvector of lambda[..., j].
    """
    return _TridiagonalEigh.apply(d, e, leaf_size, gemm_mode)


class BatchedSolver:
    """A batch of tridiagonals of fixed sizes, planned once and launched many times.

    ``prepare`` uploads the plan; ``launch`` enqueues the kernels only, so it can
    be captured with ``capture()`` into a HIP graph (torch.cuda.CUDAGraph) and
    replayed: each replay solves for the current contents of ``self.d``/``self.e``.
    """

    def __init__(self, sizes, o: Opts | None = None, device="cuda"):
        lib = load()
        self.o = o or opts()
        self.sizes = [int(x) for x in sizes]
        B = len(self.sizes)
        self.B = B
        off, qoff, acc, qacc, eacc = [], [], 0, 0, 0
        for nb_ in self.sizes:
            off.append(acc)
            qoff.append(qacc)
            acc += nb_
            qacc += nb_ * nb_
            eacc += max(nb_ - 1, 0)
        self.off, self.qoff = off, qoff
        self._n = (ctypes.c_int64 * max(B, 1))(*self.sizes)
        self._off = (ctypes.c_int64 * max(B, 1))(*off)
        self._qoff = (ctypes.c_int64 * max(B, 1))(*qoff)
        self.d = torch.zeros(max(acc, 1), dtype=torch.float64, device=device)
        self.e = torch.zeros(max(eacc, 1), dtype=torch.float64, device=device)
        self.lam = torch.empty(max(acc, 1), dtype=torch.float64, device=device)
        self.Q = torch.empty(max(qacc, 1), dtype=torch.float64, device=device)
        nb = ctypes.c_size_t()
        _check(lib.phdc_stedc_batched_workspace(B, self._n, ctypes.byref(self.o), ctypes.byref(nb)),
               "phdc_stedc_batched_workspace")
        self.work = workspace(nb.value, device)
        self.graph = None

    def prepare(self, stream=None):
        _check(load().phdc_stedc_batched_prepare(self.B, self._n, self._off, self._qoff, _ptr(self.d), _ptr(self.e),
                                                 _ptr(self.lam), _ptr(self.Q), _ptr(self.work), self.work.numel(),
                                                 ctypes.byref(self.o), _stream(stream)),
               "phdc_stedc_batched_prepare")

    def launch(self, stream=None):
        _check(load().phdc_launch_prepared(_ptr(self.work), _stream(stream)), "phdc_launch_prepared")

    def capture(self):
        """Capture ``launch`` into a HIP graph (after ``prepare``)."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            self.launch()
        torch.cuda.current_stream().wait_stream(s)
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
