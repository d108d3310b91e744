"""Plain FP64 CPU oracle for the tridiagonal divide-and-conquer eigensolver.

TEST INFRASTRUCTURE ONLY.  This package is the reference the HIP library is
checked against.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import it; the library itself never does.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc and OpenMP); this
module only marshals numpy arrays through ctypes.  See ``oracle.c`` for the
paper passages each routine follows (arXiv 1612.07526, Sec. 1, Eq. (1)-(6)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(src: str = _SRC, out: str = _LIB, extra: tuple = ()) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE: no fast-math)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-fno-fast-math",
           "-ffp-contract=off", *extra, "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def _load(path: str | None = None):
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    i, d = ctypes.c_int, ctypes.c_double
    lib.or_jacobi.argtypes = [i, _dp, i, _dp, _dp, i]
    lib.or_secular.argtypes = [i, _dp, _dp, d, _ip, _dp]
    lib.or_lowner.argtypes = [i, _dp, d, _ip, _dp, _dp, _dp]
    lib.or_lowner.restype = None
    lib.or_uhat.argtypes = [i, _dp, _ip, _dp, _dp, _dp, i]
    lib.or_uhat.restype = None
    lib.or_merge.argtypes = [i, i, _dp, _dp, d, _dp, i, _dp, i, _dp, _dp, i, _ip]
    lib.or_stedc.argtypes = [i, _dp, _dp, _dp, _dp, i, i, _ip]
    lib.or_adjoint.argtypes = [i, _dp, _dp, i, _dp, _dp, i, _dp, _dp]
    lib.or_adjoint.restype = None
    lib.or_gemm.argtypes = [i, i, i, _dp, i, _dp, i, _dp, i]
    lib.or_gemm.restype = None
    return lib


def _f64(a) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _pi(a: np.ndarray):
    return a.ctypes.data_as(_ip)


class Oracle:
    """Thin ctypes facade; ``lib`` may point at a differently compiled build."""

    def __init__(self, lib_path: str | None = None):
        self.lib = _load(lib_path)

    def jacobi(self, A):
        A = _f64(A).copy(order="F")
        n = A.shape[0]
        w = np.zeros(n)
        V = np.zeros((n, n), order="F")
        sweeps = self.lib.or_jacobi(n, _p(A), max(n, 1), _p(w), _p(V), max(n, 1))
        if sweeps < 0:
            raise RuntimeError("Jacobi did not converge")
        return w, V

    def secular(self, d, z, rho):
        d = np.ascontiguousarray(d, dtype=np.float64)
        z = np.ascontiguousarray(z, dtype=np.float64)
        K = d.size
        o = np.zeros(K, dtype=np.int32)
        tau = np.zeros(K)
        self.lib.or_secular(K, _p(d), _p(z), float(rho), _pi(o), _p(tau))
        return o, tau

    def lowner(self, d, rho, o, tau, z):
        d = np.ascontiguousarray(d, dtype=np.float64)
        z = np.ascontiguousarray(z, dtype=np.float64)
        o = np.ascontiguousarray(o, dtype=np.int32)
        tau = np.ascontiguousarray(tau, dtype=np.float64)
        zh = np.zeros(d.size)
        self.lib.or_lowner(d.size, _p(d), float(rho), _pi(o), _p(tau), _p(z), _p(zh))
        return zh

    def uhat(self, d, o, tau, zhat):
        d = np.ascontiguousarray(d, dtype=np.float64)
        o = np.ascontiguousarray(o, dtype=np.int32)
        tau = np.ascontiguousarray(tau, dtype=np.float64)
        zhat = np.ascontiguousarray(zhat, dtype=np.float64)
        K = d.size
        U = np.zeros((K, K), order="F")
        self.lib.or_uhat(K, _p(d), _pi(o), _p(tau), _p(zhat), _p(U), max(K, 1))
        return U

    def merge(self, D, z, rho, Q1, Q2):
        Q1 = _f64(Q1)
        Q2 = _f64(Q2)
        n1, n2 = Q1.shape[0], Q2.shape[0]
        D = np.ascontiguousarray(D, dtype=np.float64)
        z = np.ascontiguousarray(z, dtype=np.float64)
        m = n1 + n2
        lam = np.zeros(m)
        Q = np.zeros((m, m), order="F")
        stats = np.zeros(8, dtype=np.int32)
        self.lib.or_merge(n1, n2, _p(D), _p(z), float(rho), _p(Q1), max(n1, 1), _p(Q2), max(n2, 1),
                          _p(lam), _p(Q), max(m, 1), _pi(stats))
        return lam, Q, stats

    def stedc(self, d, e, leaf: int = 32):
        d = np.ascontiguousarray(d, dtype=np.float64)
        n = d.size
        e = np.ascontiguousarray(e, dtype=np.float64) if n > 1 else np.zeros(1)
        lam = np.zeros(n)
        Q = np.zeros((n, n), order="F")
        stats = np.zeros(8, dtype=np.int32)
        info = self.lib.or_stedc(n, _p(d), _p(e), _p(lam), _p(Q), max(n, 1), int(leaf), _pi(stats))
        if info != 0:
            raise RuntimeError(f"oracle stedc info={info}")
        return lam, Q, stats

    def adjoint(self, lam, Q, lbar, Qbar):
        Q = _f64(Q)
        Qbar = _f64(Qbar)
        n = Q.shape[0]
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        lbar = np.ascontiguousarray(lbar, dtype=np.float64)
        dbar = np.zeros(n)
        ebar = np.zeros(max(n - 1, 1))
        self.lib.or_adjoint(n, _p(lam), _p(Q), n, _p(lbar), _p(Qbar), n, _p(dbar), _p(ebar))
        return dbar, ebar[: max(n - 1, 0)]

    def gemm(self, A, B):
        A = _f64(A)
        B = _f64(B)
        m, k = A.shape
        n = B.shape[1]
        C = np.zeros((m, n), order="F")
        self.lib.or_gemm(m, n, k, _p(A), max(m, 1), _p(B), max(k, 1), _p(C), max(m, 1))
        return C


_default = None


def get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
