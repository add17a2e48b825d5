"""The C-ABI library: loads, exports every symbol of include/messi.h, and its
host-side logic (breakpoints, argument checks) behaves, all without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "messi.h")
LIB = os.path.join(ROOT, "paper_2110_07519_amd", "libmessi.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libmessi.so not built")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(messi_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    import paper_2110_07519_amd as pm

    names = declared_functions()
    assert len(names) >= 11
    L = ctypes.CDLL(LIB)
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(pm.EXPORTS)


def test_library_breakpoints_equal_oracle_bitwise():
    """The library computes its table by a different method (rational
    approximation + Halley steps); the two must agree to the last bit."""
    import paper_2110_07519_amd as pm

    for cb in range(1, 9):
        a = pm.messi_breakpoints(cb)
        b = oracle.breakpoints(cb)
        assert a.dtype == np.float32 and np.array_equal(a.view(np.uint32), b.view(np.uint32)), cb


def test_argument_checks_without_gpu():
    import paper_2110_07519_amd as pm

    L = pm.lib()
    h = ctypes.c_void_p()
    P = ctypes.c_void_p
    # null series, bad sizes: rejected before any device work
    assert L.messi_build(None, 10, 256, 16, 256, 10, ctypes.byref(h)) == pm.MESSI_EINVAL
    assert L.messi_build(P(8), 0, 256, 16, 256, 10, ctypes.byref(h)) == pm.MESSI_EINVAL
    assert L.messi_build(P(8), 10, 250, 16, 256, 10, ctypes.byref(h)) == pm.MESSI_EINVAL
    assert L.messi_build(P(8), 10, 256, 17, 256, 10, ctypes.byref(h)) == pm.MESSI_EINVAL
    assert L.messi_build(P(8), 10, 256, 16, 100, 10, ctypes.byref(h)) == pm.MESSI_EINVAL
    assert L.messi_build(P(8), 10, 256, 16, 512, 10, ctypes.byref(h)) == pm.MESSI_EINVAL
    assert L.messi_build(P(8), 10, 256, 16, 256, 0, ctypes.byref(h)) == pm.MESSI_EINVAL
    assert b"cardinality" in L.messi_last_error() or len(L.messi_last_error()) > 0
    # host pointer where a device pointer is required
    buf = np.zeros((10, 256), np.float32)
    assert L.messi_build(buf.ctypes.data_as(P), 10, 256, 16, 256, 10, ctypes.byref(h)) == pm.MESSI_EINVAL
    assert b"device" in L.messi_last_error()
    assert L.messi_query(None, None, 1, 1, 0, 0, None, None) == pm.MESSI_EINVAL
    assert L.messi_breakpoints(0, None) == pm.MESSI_EINVAL
    assert L.messi_breakpoints(9, buf.ctypes.data_as(P)) == pm.MESSI_EINVAL


def test_binding_raises_when_library_missing(monkeypatch, tmp_path):
    import paper_2110_07519_amd as pm

    monkeypatch.setattr(pm, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pm, "_lib", None)
    with pytest.raises(RuntimeError):
        pm.lib()
