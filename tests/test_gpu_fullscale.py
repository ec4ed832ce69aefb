"""Full-size parity: the 95,417,114-record library of the paper (Section 2.2)
with the paper's three strides, in the launch configurations the benchmark
times.  The oracle checks a sample of queries one by one (threaded chunk and
merge form); every query is additionally checked across the three scan paths
and against properties that hold at any size."""
import os

import numpy as np
import pytest

import fpsynth
import oracle

fps = pytest.importorskip("paper_1906_06170_amd")
torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
NTH = max(1, min(16, os.cpu_count() or 1))


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def paper_lib():
    say("generating 95,417,114 records")
    lib_np = fpsynth.make_library(fpsynth.PAPER_N, 1, keep_meta=False)
    lib = fps.Library(lib_np.words, strides=fpsynth.PAPER_STRIDES)
    yield lib_np, lib
    lib.close()


def oracle_one(lib_np, q, k, mask=None):
    rr = oracle.mask_ranges(fpsynth.PAPER_STRIDES, mask)
    return oracle.search(lib_np.words, q, k, ranges=rr, nthreads=NTH)


def properties(hits, off, k, masks, strides):
    nq = len(off) - 1
    for i in range(nq):
        h = hits[int(off[i]):int(off[i + 1])]
        m = None if masks is None else int(masks[i])
        neff = sum(e - b for b, e in oracle.mask_ranges(strides, m))
        kk = int(k if np.ndim(k) == 0 else k[i])
        assert len(h) == min(kk, neff)
        key = h["distance"].astype(np.uint64) << np.uint64(32) | h["index"].astype(np.uint64)
        assert np.all(np.diff(key.astype(np.int64)) > 0)  # strictly ascending (d, index)
        if m is not None:
            ok = np.zeros(len(h), dtype=bool)
            for b, e in oracle.mask_ranges(strides, m):
                ok |= (h["index"] >= b) & (h["index"] < e)
            assert ok.all()


def test_single_query_full(paper_lib):
    lib_np, lib = paper_lib
    qs = fpsynth.make_queries(lib_np, 4, 1001, flips=(0, 5))
    for i in range(4):
        say("case: full single query", i)
        got = lib.search(qs.words[i], 30)
        assert got["distance"][0] <= qs.flips[i]
        want = oracle_one(lib_np, qs.words[i], 30)
        assert np.array_equal(got, want), i
        assert lib.last_stats()["fallbacks"] == 0


def test_batch_1024_full(paper_lib):
    lib_np, lib = paper_lib
    bq = fpsynth.batch_queries(lib_np, 1024, 1003)
    res = {}
    for path in (fps.PATH_MFMA_I8, fps.PATH_MFMA_F4, fps.PATH_POPCOUNT, fps.PATH_SINGLE):
        say("case: full batch 1024 path", path)
        lib.set_path(path)
        res[path] = lib.search_batch(bq.words, 30)
        assert lib.last_stats()["path"] == fps.PATH_NAMES[path]
    lib.set_path(fps.PATH_AUTO)
    h0, o0 = res[fps.PATH_MFMA_I8]
    for p in (fps.PATH_MFMA_F4, fps.PATH_POPCOUNT, fps.PATH_SINGLE):
        assert np.array_equal(o0, res[p][1]) and np.array_equal(h0, res[p][0]), p
    properties(h0, o0, 30, None, fpsynth.PAPER_STRIDES)
    for i in range(0, 1024, 2):  # library-derived queries: nearest is within the flips
        assert h0["distance"][int(o0[i])] <= bq.flips[i]
    for i in (0, 1, 2, 511, 1022, 1023):
        say("case: oracle sample", i)
        want = oracle_one(lib_np, bq.words[i], 30)
        assert np.array_equal(h0[int(o0[i]):int(o0[i + 1])], want), i


def test_uneven_4096_full(paper_lib):
    lib_np, lib = paper_lib
    uq = fpsynth.batch_queries(lib_np, 4096, 1004).words
    k, m = fpsynth.uneven_params(4096, 1004)
    res = {}
    for path in (fps.PATH_MFMA_I8, fps.PATH_MFMA_F4, fps.PATH_POPCOUNT):
        say("case: full uneven 4096 path", path)
        lib.set_path(path)
        res[path] = lib.search_batch(uq, k, m)
    lib.set_path(fps.PATH_AUTO)
    h0, o0 = res[fps.PATH_MFMA_I8]
    for p in (fps.PATH_MFMA_F4, fps.PATH_POPCOUNT):
        assert np.array_equal(o0, res[p][1]) and np.array_equal(h0, res[p][0]), p
    properties(h0, o0, k, m, fpsynth.PAPER_STRIDES)
    picks = []
    for mask in fpsynth.MASK_CHOICES:
        for kk in (1, 1000):
            idx = np.nonzero((m == mask) & (k == kk))[0]
            picks.append(int(idx[0]))
    for i in picks:
        say("case: oracle sample", i, "k", int(k[i]), "mask", int(m[i]))
        want = oracle_one(lib_np, uq[i], int(k[i]), int(m[i]))
        assert np.array_equal(h0[int(o0[i]):int(o0[i + 1])], want), i
