"""CPU checks of the ensemble server's argument validation (no device work)."""
import ctypes
import os

import pytest


def _lib():
    from paper_2605_29598_amd import binding as B
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libimexdg.so not built")
    return B, B.lib()


def test_server_create_rejects_bad_pools():
    B, L = _lib()
    h = ctypes.c_void_p()
    assert L.imx_server_create(None, 1 << 20, 2, ctypes.byref(h)) == B.IMX_EINVAL
    buf = ctypes.create_string_buffer(1 << 13)
    addr = ctypes.addressof(buf)
    unaligned = addr + (1 if addr % 256 == 0 else 0)
    assert L.imx_server_create(ctypes.c_void_p(unaligned), 4096, 2, ctypes.byref(h)) == B.IMX_EINVAL
    aligned = addr + (-addr) % 256
    assert L.imx_server_create(ctypes.c_void_p(aligned), 4096, 0, ctypes.byref(h)) == B.IMX_EINVAL
    assert L.imx_server_create(ctypes.c_void_p(aligned), 1024, 1, ctypes.byref(h)) == B.IMX_EINVAL
    assert L.imx_server_create(ctypes.c_void_p(aligned), 4096, 1, None) == B.IMX_EINVAL


def test_server_null_handles():
    B, L = _lib()
    r, w = ctypes.c_int(), ctypes.c_int()
    assert L.imx_server_tick(None, ctypes.byref(r), ctypes.byref(w)) == B.IMX_EINVAL
    assert L.imx_server_query(None, None) == B.IMX_EINVAL
    assert L.imx_server_result(None, 1, None, None) == B.IMX_EINVAL
    L.imx_server_destroy(None)
