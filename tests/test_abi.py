"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "phdc.h")


def _lib():
    import paper_1612_07526_amd as P
    if not os.path.exists(P.LIB_PATH):
        import paper_1612_07526_amd.build as B
        B.build()
    return P, P.load()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|size_t)\s+(phdc_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ["phdc_stedc", "phdc_merge", "phdc_stedc_batched", "phdc_stedc_backward", "phdc_status",
                 "phdc_secular", "phdc_opts_default", "phdc_stedc_workspace"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    P, lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), f"libphdc.so does not export {name}"


def test_version_and_defaults():
    P, lib = _lib()
    assert lib.phdc_version() >= 1
    o = P.opts()
    assert o.leaf_size == 16 and o.gemm_mode == P.GEMM_FP64 and o.hss_min_K == 4096
    assert o.hss_rel_tol == 1e-14


def test_workspace_queries_are_host_only():
    P, lib = _lib()
    o = P.opts()
    nb = ctypes.c_size_t()
    assert lib.phdc_stedc_workspace(16384, ctypes.byref(o), ctypes.byref(nb)) == 0
    # two n x n buffers' worth at least (twin eigenvector buffer + Uhat arena)
    assert nb.value >= 2 * 16384 * 16384 * 8
    assert lib.phdc_stedc_workspace(0, ctypes.byref(o), ctypes.byref(nb)) == 0
    assert lib.phdc_merge_workspace(100, 28, ctypes.byref(o), ctypes.byref(nb)) == 0
    assert nb.value >= 2 * 128 * 128 * 8
    n = (ctypes.c_int64 * 3)(5, 0, 70)
    assert lib.phdc_stedc_batched_workspace(3, n, ctypes.byref(o), ctypes.byref(nb)) == 0


@pytest.mark.parametrize("field,value", [("leaf_size", 1), ("leaf_size", 65), ("gemm_mode", 7), ("hss_leaf", 4),
                                         ("hss_leaf", 2048), ("hss_samples", 8), ("hss_samples", 1024),
                                         ("hss_samples_inc", -1), ("hss_rel_tol", 0.0), ("hss_rel_tol", 1.5),
                                         ("split_slices", 0), ("split_slices", 8)])
def test_bad_options_rejected(field, value):
    P, lib = _lib()
    o = P.opts(**{field: value})
    nb = ctypes.c_size_t()
    assert lib.phdc_stedc_workspace(100, ctypes.byref(o), ctypes.byref(nb)) == -2


def test_argument_validation_codes():
    P, lib = _lib()
    o = P.opts()
    v = ctypes.c_void_p
    fake = v(0x1000)  # never dereferenced: every call below fails its host-side checks first
    # n < 0
    assert lib.phdc_stedc(-1, fake, fake, fake, fake, 1, fake, 1 << 30, ctypes.byref(o), v(0)) == -1
    # missing d / e / lambda / Q
    assert lib.phdc_stedc(4, v(0), fake, fake, fake, 4, fake, 1 << 30, ctypes.byref(o), v(0)) == -2
    assert lib.phdc_stedc(4, fake, v(0), fake, fake, 4, fake, 1 << 30, ctypes.byref(o), v(0)) == -3
    assert lib.phdc_stedc(4, fake, fake, v(0), fake, 4, fake, 1 << 30, ctypes.byref(o), v(0)) == -4
    assert lib.phdc_stedc(4, fake, fake, fake, v(0), 4, fake, 1 << 30, ctypes.byref(o), v(0)) == -5
    # ldq < n
    assert lib.phdc_stedc(4, fake, fake, fake, fake, 3, fake, 1 << 30, ctypes.byref(o), v(0)) == -6
    # no workspace / too small
    assert lib.phdc_stedc(4, fake, fake, fake, fake, 4, v(0), 1 << 30, ctypes.byref(o), v(0)) == -7
    assert lib.phdc_stedc(4, fake, fake, fake, fake, 4, fake, 16, ctypes.byref(o), v(0)) == -8
    # merge: negative / NaN rho, bad leading dimensions
    args = lambda rho, ld1=3, ld2=2: (3, 2, fake, fake, rho, fake, ld1, fake, ld2, fake, fake, 5, fake, 1 << 30,
                                      ctypes.byref(o), v(0))
    assert lib.phdc_merge(*args(-1.0)) == -5
    assert lib.phdc_merge(*args(float("nan"))) == -5
    assert lib.phdc_merge(*args(1.0, ld1=2)) == -7
    assert lib.phdc_merge(*args(1.0, ld2=1)) == -9
    # secular: rho must be > 0
    assert lib.phdc_secular(3, fake, fake, 0.0, fake, fake, fake, 256, v(0)) == -4
    # batched: offsets must be the prefix sums of the sizes
    n = (ctypes.c_int64 * 2)(3, 4)
    off = (ctypes.c_int64 * 2)(0, 2)
    qoff = (ctypes.c_int64 * 2)(0, 9)
    assert lib.phdc_stedc_batched(2, n, off, qoff, fake, fake, fake, fake, fake, 1 << 30, ctypes.byref(o),
                                  v(0)) == -3


def test_autotune_workspace_checks():
    P, lib = _lib()
    nb = ctypes.c_size_t()
    assert lib.phdc_autotune_gemm_workspace(4096, ctypes.byref(nb)) == 0
    assert nb.value >= 3 * 4096 * 4096 * 8
    assert lib.phdc_autotune_gemm_workspace(1, ctypes.byref(nb)) == -1
    assert lib.phdc_autotune_gemm_workspace((1 << 20) + 1, ctypes.byref(nb)) == -1
    assert lib.phdc_autotune_gemm(4096, None, 0, None) == -2
    tiles = (ctypes.c_int32 * 32)()
    assert lib.phdc_gemm_tile_table(tiles, 32) == 21
