"""Full-size parity: the 95,417,114-record library of the paper (Section 2.2)
with the paper's three strides, in the launch configurations the benchmark
times.  Every query of the full-size workloads is compared with the expected
results the CPU oracle wrote (tests/golden/make_fullscale.py: the threaded
chunk-and-merge form of oracle.c, Fig. 3 top-k of the Section 4.3 distance):

  * the 32 headline single queries (seed 1001): the whole top-30, every entry;
  * the 1,024-query batch (seed 1003): the whole top-30 of every query on every
    scan path, and the 16-byte SHA-256 prefix of every top-100 and top-1,000;
  * the 4,096-query uneven batch (seed 1004, per-query k and stride masks):
    the hash of every result list, on every batched path;
  * requests served at full size (k in {30, 100, 1000}), alone and in the mix.

The library is checked first against the SHA-256 of its words recorded with
the expected values, so a change of the generator cannot pass silently."""
import hashlib
import json
import os

import numpy as np
import pytest

import fpsynth
import oracle

fps = pytest.importorskip("paper_1906_06170_amd")
torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullscale_95M")
BATCH_PATHS = (fps.PATH_MFMA_I8, fps.PATH_MFMA_F4, fps.PATH_POPCOUNT)


def say(*a):
    print(*a, flush=True)


def hit_hash(h) -> bytes:
    """First 16 bytes of SHA-256 over the (uint32 index, uint32 distance)
    little-endian pairs of a result list (the rule of make_fullscale.py)."""
    a = np.empty((len(h), 2), dtype="<u4")
    a[:, 0] = h["index"]
    a[:, 1] = h["distance"]
    return hashlib.sha256(a.tobytes()).digest()[:16]


@pytest.fixture(scope="module")
def gold():
    meta = json.load(open(GOLDEN + ".json"))
    z = dict(np.load(GOLDEN + ".npz", allow_pickle=False))
    return meta, z


@pytest.fixture(scope="module")
def paper_lib(gold):
    meta, _ = gold
    say("generating 95,417,114 records")
    lib_np = fpsynth.make_library(fpsynth.PAPER_N, 1, keep_meta=False)
    digest = hashlib.sha256(np.ascontiguousarray(lib_np.words, dtype="<u8").tobytes()).hexdigest()
    assert digest == meta["library"]["words_sha256"], "the generator no longer makes this library"
    assert meta["library"]["strides"] == list(fpsynth.PAPER_STRIDES)
    lib = fps.Library(lib_np.words, strides=fpsynth.PAPER_STRIDES)
    yield lib_np, lib
    lib.close()


def queries_sha(words) -> str:
    return hashlib.sha256(np.ascontiguousarray(words, dtype="<u8").tobytes()).hexdigest()


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


def test_single_queries_all_equal_the_oracle(paper_lib, gold):
    meta, z = gold
    lib_np, lib = paper_lib
    nq = meta["single"]["nq"]
    qs = fpsynth.make_queries(lib_np, nq, meta["single"]["seed"], flips=(0, 5))
    assert queries_sha(qs.words) == meta["single"]["queries_sha256"]
    for i in range(nq):
        say("case: full single query", i)
        got = lib.search(qs.words[i], 30)
        assert len(got) == int(z["single_count"][i]) == 30
        assert np.array_equal(got["index"], z["single_index"][i]), i
        assert np.array_equal(got["distance"], z["single_distance"][i]), i
        assert got["distance"][0] <= qs.flips[i]
        assert lib.last_stats()["fallbacks"] == 0


def test_batch_1024_every_query_every_path(paper_lib, gold):
    meta, z = gold
    lib_np, lib = paper_lib
    bq = fpsynth.batch_queries(lib_np, 1024, meta["batch"]["seed"])
    assert queries_sha(bq.words) == meta["batch"]["queries_sha256"]
    for path in BATCH_PATHS + (fps.PATH_SINGLE,):
        say("case: full batch 1024 top-30 path", fps.PATH_NAMES[path])
        lib.set_path(path)
        h, o = lib.search_batch(bq.words, 30)
        assert lib.last_stats()["path"] == fps.PATH_NAMES[path]
        properties(h, o, 30, None, fpsynth.PAPER_STRIDES)
        idx = h["index"].reshape(1024, 30)
        dist = h["distance"].reshape(1024, 30)
        bad = np.nonzero(~(np.all(idx == z["batch_index"], axis=1)
                           & np.all(dist == z["batch_distance"], axis=1)))[0]
        assert len(bad) == 0, f"{fps.PATH_NAMES[path]}: queries {bad[:10]} differ"
    lib.set_path(fps.PATH_AUTO)
    for k, key in ((100, "batch_top100_hash"), (1000, "batch_top1000_hash")):
        for path in (fps.PATH_MFMA_F4, fps.PATH_POPCOUNT):
            say("case: full batch 1024 top", k, "path", fps.PATH_NAMES[path])
            lib.set_path(path)
            h, o = lib.search_batch(bq.words, k)
            bad = [i for i in range(1024)
                   if hit_hash(h[int(o[i]):int(o[i + 1])]) != bytes(z[key][i])]
            assert not bad, f"top-{k} {fps.PATH_NAMES[path]}: queries {bad[:10]} differ"
            if k == 1000:
                assert np.array_equal(h["distance"][o[1:].astype(np.int64) - 1],
                                      z["batch_last1000"])
    lib.set_path(fps.PATH_AUTO)


def test_uneven_4096_every_query_every_path(paper_lib, gold):
    meta, z = gold
    lib_np, lib = paper_lib
    uq = fpsynth.batch_queries(lib_np, 4096, meta["uneven"]["seed"]).words
    k, m = fpsynth.uneven_params(4096, meta["uneven"]["seed"])
    assert queries_sha(uq) == meta["uneven"]["queries_sha256"]
    assert hashlib.sha256(k.astype("<u4").tobytes()).hexdigest() == meta["uneven"]["k_sha256"]
    assert hashlib.sha256(m.astype("<u4").tobytes()).hexdigest() == meta["uneven"]["mask_sha256"]
    for path in BATCH_PATHS:
        say("case: full uneven 4096 path", fps.PATH_NAMES[path])
        lib.set_path(path)
        h, o = lib.search_batch(uq, k, m)
        properties(h, o, k, m, fpsynth.PAPER_STRIDES)
        assert np.array_equal(np.diff(o).astype(np.uint32), z["uneven_count"])
        bad = [i for i in range(4096)
               if hit_hash(h[int(o[i]):int(o[i + 1])]) != bytes(z["uneven_hash"][i])]
        assert not bad, f"{fps.PATH_NAMES[path]}: queries {bad[:10]} differ"
    lib.set_path(fps.PATH_AUTO)


def test_served_requests_alone_and_in_the_mix(paper_lib, gold):
    """A few hundred requests of the 1,024-query batch (1-64 queries each, k in
    {30, 100, 1000}) served at full size: each request's results equal the
    oracle's (expected arrays and hashes), whether it is served alone or
    coalesced with the others."""
    meta, z = gold
    lib_np, lib = paper_lib
    bq = fpsynth.batch_queries(lib_np, 1024, meta["batch"]["seed"]).words
    rng = np.random.default_rng(77)
    reqs = []
    for _ in range(300):
        size = int(rng.integers(1, 65))
        reqs.append((int(rng.integers(0, 1024 - size + 1)), size, int(rng.choice([30, 100, 1000]))))

    def check(first, size, k, hits, off):
        for j in range(size):
            i = first + j
            h = hits[int(off[j]):int(off[j + 1])]
            if k == 30:
                assert np.array_equal(h["index"], z["batch_index"][i]), i
                assert np.array_equal(h["distance"], z["batch_distance"][i]), i
            else:
                key = "batch_top100_hash" if k == 100 else "batch_top1000_hash"
                assert hit_hash(h) == bytes(z[key][i]), (i, k)

    srv = fps.Server(lib, pool_bytes=4 << 30, max_batch_queries=512, n_streams=3,
                     reserve_streams=1)
    say("case: served alone", len(reqs))
    for first, size, k in reqs[:40]:
        t = srv.submit(bq[first:first + size], k)
        hits, off, _ = srv.wait(t)
        check(first, size, k, hits, off)
    say("case: served in the mix", len(reqs))
    tickets = [srv.submit(bq[first:first + size], k) for first, size, k in reqs]
    batched = 0
    for (first, size, k), t in zip(reqs, tickets):
        hits, off, st = srv.wait(t)
        check(first, size, k, hits, off)
        batched += st["batch_queries"] > size
    assert batched > 0, "no request was coalesced with others"
    srv.close()
