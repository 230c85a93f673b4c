"""The C-ABI library loads on a machine without a GPU and exports every entry
point that include/fftnk.h declares (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "fftnk.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fftnk_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_1603_08893_amd import fftnk
    path = fftnk._LIB_PATH
    if not os.path.exists(path):
        pytest.skip("libfftnk.so not built")
    L = ctypes.CDLL(path)
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert sorted(fftnk.EXPORTS) == names


def test_status_strings_and_argument_checks():
    from paper_1603_08893_amd import fftnk
    if not os.path.exists(fftnk._LIB_PATH):
        pytest.skip("libfftnk.so not built")
    L = fftnk.lib()
    assert L.fftnk_status_string(0) == b"ok"
    assert b"CG" in L.fftnk_status_string(fftnk.ECG_MAXIT)
    ctx = ctypes.c_void_p()
    # invalid sizes are rejected on the host, before any device work
    assert L.fftnk_create(ctypes.byref(ctx), 1, 8, 8, 0, None) == fftnk.EINVAL
    # axis limits: a0 / a1 up to 512, a2 up to 256
    assert L.fftnk_create(ctypes.byref(ctx), 513, 8, 8, 0, None) == fftnk.EUNSUPPORTED
    assert L.fftnk_create(ctypes.byref(ctx), 8, 600, 8, 0, None) == fftnk.EUNSUPPORTED
    assert L.fftnk_create(ctypes.byref(ctx), 8, 8, 257, 0, None) == fftnk.EUNSUPPORTED
    assert L.fftnk_create(ctypes.byref(ctx), 8, 8, 300, 0, None) == fftnk.EUNSUPPORTED
    assert L.fftnk_create(ctypes.byref(ctx), 8, 8, 8, 7, None) == fftnk.EINVAL
