"""The allocation-free single-query search (fps_search_noalloc) against the
search with a caller-owned workspace (fps_search), bit-exactly, through the C
ABI: two calls in a row, the second with a smaller input, then a search too
large for the static scratch, which must be refused."""
import ctypes

import numpy as np
import pytest

import fpsynth
import oracle

fps = pytest.importorskip("paper_1906_06170_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def noalloc(lib, q, k, mask):
    c = fps.load_library()
    q = np.ascontiguousarray(np.asarray(q, dtype=np.uint64).reshape(3))
    out = np.empty(max(int(k), 1), dtype=fps.HIT_DTYPE)
    n = ctypes.c_uint32()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = c.fps_search_noalloc(lib.handle, ctypes.c_void_p(q.ctypes.data), int(k), int(mask),
                              ctypes.c_void_p(out.ctypes.data), ctypes.byref(n), stream)
    return rc, out[:n.value].copy()


def test_noalloc_matches_workspace_search():
    lib_np = fpsynth.make_library(100_000, 3)
    lib = fps.Library(lib_np.words, strides=[0, 40_000, 75_000, 100_000])
    qs = fpsynth.batch_queries(lib_np, 4, 91).words
    try:
        # two calls in a row, the second smaller (fewer results, one stride)
        for q, k, mask in ((qs[0], 1000, fps.MASK_ALL), (qs[1], 10, 0b001),
                           (qs[2], 30, 0b110), (qs[3], 0, fps.MASK_ALL)):
            say("case: noalloc k", k, "mask", mask)
            rc, got = noalloc(lib, q, k, mask)
            assert rc == fps.FPS_OK, fps.load_library().fps_last_error()
            want = lib.search(q, k, mask)
            assert np.array_equal(got, want)
            ranges = oracle.mask_ranges(lib.strides, None if mask == fps.MASK_ALL else mask)
            assert np.array_equal(got, oracle.search(lib_np.words, q, k, ranges=ranges))
    finally:
        lib.close()


def test_noalloc_refuses_beyond_its_scratch():
    n = 4_000_000
    lib_np = fpsynth.make_library(n, 4, keep_meta=False)
    lib = fps.Library(lib_np.words)
    q = fpsynth.batch_queries(lib_np, 1, 92).words[0]
    try:
        say("case: noalloc over its scratch")
        rc, _ = noalloc(lib, q, n, fps.MASK_ALL)
        assert rc == fps.FPS_E_NOMEM
        assert b"static scratch" in fps.load_library().fps_last_error()
        # a search that fits still works afterwards, and agrees with fps_search
        rc, got = noalloc(lib, q, 30, fps.MASK_ALL)
        assert rc == fps.FPS_OK
        assert np.array_equal(got, lib.search(q, 30))
    finally:
        lib.close()
