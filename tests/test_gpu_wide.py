"""Wider fingerprints (Section 5, concluding remark 3) on the GPU against the
oracle's width-generic key loop: 256-, 1,024- and 2,048-key libraries, every
scan path (single, popcount, int8 and fp4 matrix cores), uneven k, stride
masks, ragged strides, ties, several scan phases, the overflow fallback and
k edges.  Integer results: bit-exact (ids, distances, order)."""
import numpy as np
import pytest

import fpsynth
import oracle

fps = pytest.importorskip("paper_1906_06170_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

PATHS = [fps.PATH_SINGLE, fps.PATH_POPCOUNT, fps.PATH_MFMA_I8, fps.PATH_MFMA_F4]


def say(*a):
    print(*a, flush=True)


_cache = {}


def setup(W, n=50_021, seed=3):
    key = (W, n, seed)
    if key not in _cache:
        lib_np = fpsynth.make_wide_library(n, W, seed)
        strides = [0, n // 3 + 7, n // 2 + 1, n]
        lib = fps.WideLibrary(lib_np.words, strides=strides)
        _cache[key] = (lib_np, lib, strides)
    return _cache[key]


def check(lib_np, lib, strides, qs, k, masks, path, what):
    lib.set_path(path)
    say("case:", what, "path", fps.PATH_NAMES[path], "q", len(qs))
    hits, off = lib.search_batch(qs, k, masks)
    ohits, ooff = oracle.search_batch_w(lib_np.words, qs, k, strides, masks)
    assert np.array_equal(off, ooff), what
    for i in range(len(qs)):
        a = hits[int(off[i]):int(off[i + 1])]
        b = ohits[int(ooff[i]):int(ooff[i + 1])]
        assert np.array_equal(a, b), f"{what} {fps.PATH_NAMES[path]}: query {i}\n{a[:8]}\n{b[:8]}"
    lib.set_path(fps.PATH_AUTO)
    return lib.last_stats()


@pytest.mark.parametrize("W", [4, 16, 32])
@pytest.mark.parametrize("path", PATHS)
def test_wide_paths_uneven_k_and_masks(W, path):
    lib_np, lib, strides = setup(W)
    qs, _, _ = fpsynth.make_wide_queries(lib_np, 40, 100 + W)
    rng = np.random.default_rng(W)
    k = rng.choice(np.array([1, 10, 30, 100, 1000], dtype=np.uint32), 40)
    masks = rng.choice(np.array([1, 3, 7, 2, 4, 6], dtype=np.uint32), 40)
    st = check(lib_np, lib, strides, qs, k, masks, path, f"W={W} uneven")
    assert st["path"] == fps.PATH_NAMES[path]


@pytest.mark.parametrize("W", [4, 32])
def test_wide_k_edges(W):
    lib_np, lib, strides = setup(W)
    qs, _, _ = fpsynth.make_wide_queries(lib_np, 5, 7)
    for path in PATHS:
        for k in (0, 1, 50_020, 50_021, 60_000):
            check(lib_np, lib, strides, qs[:3], k, None, path, f"W={W} k={k}")
        check(lib_np, lib, strides, qs, [0, 5, 16_000, 3, 1], [2, 2, 2, 1, 4], path,
              f"W={W} k beyond one stride")


@pytest.mark.parametrize("path", PATHS)
def test_wide_phases_fallback_and_overflow(path):
    lib_np, lib, strides = setup(16)
    qs, _, _ = fpsynth.make_wide_queries(lib_np, 12, 55)
    k = np.array([1, 30, 100, 1000] * 3, dtype=np.uint32)
    # several scan phases: a small bound sample
    lib.set_tuning(sample_records=512)
    check(lib_np, lib, strides, qs, k, None, path, "phases")
    # the exact fallback for every query, and forced buffer overflows
    lib.set_tuning(force_fallback=True)
    st = check(lib_np, lib, strides, qs, k, None, path, "forced fallback")
    assert st["fallbacks"] == 12
    lib.set_tuning(candidate_scale=1e-4)
    st = check(lib_np, lib, strides, qs, k, None, path, "overflow")
    assert st["fallbacks"] > 0
    lib.set_tuning()


def test_wide_identical_rows_ties():
    W = 8
    row = fpsynth.make_wide_library(3, W, 1).words
    words = np.concatenate([np.tile(row[0], (30_000, 1)), np.tile(row[1], (20_000, 1))])
    cut = [0, 12_345, 30_000, 50_000]
    lib = fps.WideLibrary(words, strides=cut)
    q = row[0].copy()
    q[0] ^= np.uint64(1)
    for path in PATHS:
        lib.set_path(path)
        for k, mask in ((1, 7), (30, 2), (5000, 3), (29_999, 7)):
            h = lib.search(q, k, mask)
            rr = oracle.mask_ranges(cut, mask)
            assert np.array_equal(h, oracle.search_w(words, q, k, rr)), (path, k, mask)


def test_wide_argument_errors():
    w = np.zeros((10, 3), dtype=np.uint64)
    with pytest.raises(fps.FPSError):
        fps.WideLibrary(w)
    lib_np, lib, strides = setup(4)
    with pytest.raises(fps.FPSError):
        lib.search_batch(np.zeros((1, 4), dtype=np.uint64), [3], [8])
