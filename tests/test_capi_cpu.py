"""The C-ABI library loads without a GPU, exports every entry point that
include/fps.h declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1906_06170_amd as fps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fps.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fps_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fps.SO_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return fps.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = header_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(fps.EXPORTS), set(names) ^ set(fps.EXPORTS)


def test_device_bytes_layout(lib):
    assert lib.fps_library_device_bytes(1) == 4096 * 21
    assert lib.fps_library_device_bytes(4096) == 4096 * 21
    assert lib.fps_library_device_bytes(4097) == 8192 * 21
    assert lib.fps_library_device_bytes(95_417_114) == 95_420_416 * 21


def test_host_side_errors(lib):
    w = np.zeros((4, 3), dtype=np.uint64)
    h = ctypes.c_void_p()
    rc = lib.fps_library_load(None, 4, None, 0, None, 0, None, ctypes.byref(h))
    assert rc == fps.FPS_E_ARG and b"NULL" in lib.fps_last_error()
    dummy = ctypes.c_void_p(256)  # never dereferenced: validation fails first
    rc = lib.fps_library_load(ctypes.c_void_p(w.ctypes.data), 0, None, 0, dummy, 1 << 20, None,
                              ctypes.byref(h))
    assert rc == fps.FPS_E_ARG
    rc = lib.fps_library_load(ctypes.c_void_p(w.ctypes.data), 4, None, 0, dummy, 100, None,
                              ctypes.byref(h))
    assert rc == fps.FPS_E_ARG and b"device buffer" in lib.fps_last_error()
    w[2, 0] = 1  # bit 0 set
    rc = lib.fps_library_load(ctypes.c_void_p(w.ctypes.data), 4, None, 0, dummy, 1 << 20, None,
                              ctypes.byref(h))
    assert rc == fps.FPS_E_FINGERPRINT and b"record 2" in lib.fps_last_error()
    w[2, 0] = 0
    w[1, 2] = np.uint64(1) << np.uint64(39)  # key 167
    rc = lib.fps_library_load(ctypes.c_void_p(w.ctypes.data), 4, None, 0, dummy, 1 << 20, None,
                              ctypes.byref(h))
    assert rc == fps.FPS_E_FINGERPRINT and b"record 1" in lib.fps_last_error()
    st = np.array([0, 3, 2, 4], dtype=np.uint64)
    w[1, 2] = 0
    rc = lib.fps_library_load(ctypes.c_void_p(w.ctypes.data), 4, ctypes.c_void_p(st.ctypes.data),
                              3, dummy, 1 << 20, None, ctypes.byref(h))
    assert rc == fps.FPS_E_ARG and b"decrease" in lib.fps_last_error()
    assert lib.fps_search(None, None, 1, 1, None, 0, None, None, None) == fps.FPS_E_ARG
    assert lib.fps_search_batch(None, None, 1, None, None, None, 0, None, 0, None,
                                None) == fps.FPS_E_ARG
    sz = ctypes.c_size_t()
    assert lib.fps_workspace_bytes(None, 1, None, None, ctypes.byref(sz)) == fps.FPS_E_ARG
    assert lib.fps_set_tuning(None, 1.0, 0, 0, 0) == fps.FPS_E_ARG
    assert lib.fps_set_path(None, 0) == fps.FPS_E_ARG
    assert lib.fps_library_free(None) == fps.FPS_OK
    assert lib.fps_server_destroy(None) == fps.FPS_OK
    assert lib.fps_last_error() == b""


def test_binding_fails_loudly_without_gpu(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError):
        fps.Library(np.zeros((8, 3), dtype=np.uint64))
