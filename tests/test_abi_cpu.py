"""Host-side checks of the C ABI (no GPU): exported symbols, defaults, argument and geometry errors.

The library's argument validation and contact search run before any HIP call, so
these error paths are exercised on the CPU.
"""

import ctypes as C
import json
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "mfs.h")
LIB = os.path.join(ROOT, "paper_2606_11273_amd", "libmfs_hip.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libmfs_hip.so not built (run __graft_entry__.build())")


def _declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mfs_[a-z_0-9]+)\s*\(", txt)))


def _lib():
    import torch  # noqa: F401  (same HIP runtime as the binding)
    from paper_2606_11273_amd import native
    return native, native.lib()


def test_every_declared_symbol_is_exported():
    native, L = _lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert sorted(native.SYMBOLS) == names


def test_default_params_are_the_papers():
    native, _ = _lib()
    p = native.mfs_default_params()
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_parameters.json")))
    for k in ("delta_c", "eps_ring", "n_fp", "n_ell", "m_p", "eps_trunc", "eps_trunc_fine", "gamma", "a_f",
              "mobius_r", "a_ell"):
        assert getattr(p, k) == gold[k]["value"], k
    assert p.mu == 1.0


def test_setup_rejects_bad_arguments_and_overlaps_without_touching_the_device():
    native, L = _lib()
    ctx = C.c_void_p()
    c = np.array([[0.0, 0.0], [2.5, 0.0]])
    a = np.ones(2)
    ns = np.full(2, 36, dtype=np.int32)
    nc = np.full(2, 72, dtype=np.int32)
    rs = np.full(2, 0.7)
    dp = lambda x: x.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    ip = lambda x: x.ctypes.data_as(C.POINTER(C.c_int32))  # noqa: E731
    assert L.mfs_setup(C.byref(ctx), 0, dp(c), dp(a), ip(ns), ip(nc), dp(rs), None, None) == native.MFS_ERR_ARG
    bad = nc.copy()
    bad[1] = 30
    assert L.mfs_setup(C.byref(ctx), 2, dp(c), dp(a), ip(ns), ip(bad), dp(rs), None, None) == native.MFS_ERR_ARG
    assert b"n_src" in L.mfs_last_error(None)
    over = np.array([[0.0, 0.0], [1.9, 0.0]])
    assert L.mfs_setup(C.byref(ctx), 2, dp(over), dp(a), ip(ns), ip(nc), dp(rs), None, None) == native.MFS_ERR_GEOMETRY
    assert b"overlap" in L.mfs_last_error(None)
    touch = np.array([[0.0, 0.0], [2.0, 0.0]])
    assert L.mfs_setup(C.byref(ctx), 2, dp(touch), dp(a), ip(ns), ip(nc), dp(rs), None, None) == native.MFS_ERR_GEOMETRY
    p = native.mfs_default_params()
    p.gamma = 1.5
    assert L.mfs_setup(C.byref(ctx), 2, dp(c), dp(a), ip(ns), ip(nc), dp(rs), C.byref(p), None) == native.MFS_ERR_ARG
    assert not ctx.value
    assert L.mfs_destroy(None) == native.MFS_OK


def test_server_rejects_bad_arguments_without_touching_the_device():
    native, L = _lib()
    srv = C.c_void_p()
    assert L.mfs_server_create(C.byref(srv), 0, 0, None) == native.MFS_ERR_ARG
    assert L.mfs_server_create(C.byref(srv), 0, 65, None) == native.MFS_ERR_ARG
    assert L.mfs_server_create(None, 0, 1, None) == native.MFS_ERR_ARG
    assert not srv.value
    out = np.zeros(3)
    assert L.mfs_server_wait(None, 1, out.ctypes.data_as(C.POINTER(C.c_double)), None, 0) == native.MFS_ERR_ARG
    assert L.mfs_server_destroy(None) == native.MFS_OK
