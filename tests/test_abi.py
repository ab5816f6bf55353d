"""The C-ABI library loads and exports every symbol include/fdwt.h declares
(no device calls; runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_0808_0487_amd import fdwt

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "fdwt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdwt_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["fdwt_net_generate", "fdwt_dwt_forward", "fdwt_dwt_inverse", "fdwt_walsh_interp", "fdwt_eff_dim"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(fdwt.LIB_PATH):
        pytest.fail("libfdwt.so is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(fdwt.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_covers_every_declared_symbol():
    assert sorted(fdwt.SIGNATURES) == declared_functions()


def test_query_depth_without_device():
    assert fdwt.query_depth(2) == 32 and fdwt.query_depth(3) == 20 and fdwt.query_depth(5) == 13


def test_invalid_arguments_rejected_before_device_work():
    """Validation runs on the host: bad p, m, s and entries are refused with
    FDWT_EINVAL / FDWT_EUNSUPPORTED before any HIP call."""
    import numpy as np
    L = fdwt.lib()
    h = ctypes.c_void_p()
    C = np.zeros((1, 3, 3), dtype=np.uint8)
    ptr = C.ctypes.data_as(ctypes.c_void_p)
    assert L.fdwt_net_generate(4, 3, 1, ptr, ctypes.byref(h)) == fdwt.EINVAL
    assert L.fdwt_net_generate(11, 3, 1, ptr, ctypes.byref(h)) == fdwt.EUNSUPPORTED
    assert L.fdwt_net_generate(2, 0, 1, ptr, ctypes.byref(h)) == fdwt.EINVAL
    assert L.fdwt_net_generate(2, 27, 1, ptr, ctypes.byref(h)) == fdwt.EINVAL
    assert L.fdwt_net_generate(2, 3, 65, ptr, ctypes.byref(h)) == fdwt.EINVAL
    C[0, 0, 0] = 2
    assert L.fdwt_net_generate(2, 3, 1, ptr, ctypes.byref(h)) == fdwt.EINVAL
    assert b"entry" in L.fdwt_last_error()
    assert L.fdwt_dwt_forward(None, 1, None, 1, None, None) == fdwt.EINVAL
