"""GPU path vs the CPU oracle, element by element (ids, distances and order),
on seeded synthetic libraries small enough for the oracle to finish in seconds.
Integer results: the bar is bit-exact equality."""
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


@pytest.fixture(scope="module")
def small():
    lib_np = fpsynth.make_library(100_000, 1)
    strides = [0, 40_000, 75_000, 100_000]
    lib = fps.Library(lib_np.words, strides=strides)
    return lib_np, lib


def check_batch(lib_np, lib, queries, k, masks=None, path=None, what=""):
    if path is not None:
        lib.set_path(path)
    say("case:", what, "path", path, "q", len(queries))
    hits, off = lib.search_batch(queries, k, masks)
    ohits, ooff = oracle.search_batch(lib_np.words, queries, k, lib.strides, masks)
    assert np.array_equal(off, ooff), what
    if not np.array_equal(hits, ohits):
        for i in range(len(queries)):
            a = hits[int(off[i]):int(off[i + 1])]
            b = ohits[int(ooff[i]):int(ooff[i + 1])]
            assert np.array_equal(a, b), f"{what}: query {i} differs\n{a[:10]}\n{b[:10]}"
    lib.set_path(fps.PATH_AUTO)
    return lib.last_stats()


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6, 7, 8])
def test_small_single_query_seeds(seed):
    """100,000 records, a library record with 2 flips, top-30 (several seeds)."""
    lib_np, q, k, _ = fpsynth.workload_small(seed)
    lib = fps.Library(lib_np.words)
    say("case: small seed", seed)
    got = lib.search(q.words[0], 30)
    want = oracle.search(lib_np.words, q.words[0], 30)
    assert np.array_equal(got, want)
    assert got["distance"][0] <= 2
    st = lib.last_stats()
    assert st["fallbacks"] == 0 and st["path"] == "single"


@pytest.mark.parametrize("k", [0, 1, 2, 30, 1000, 8000, 99_999, 100_000, 100_007])
def test_k_edges_single(small, k):
    lib_np, lib = small
    q = fpsynth.batch_queries(lib_np, 2, 11).words[1]
    say("case: k edge", k)
    got = lib.search(q, k)
    want = oracle.search(lib_np.words, q, k)
    assert len(got) == min(k, 100_000)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("path", PATHS)
def test_batch_paths_uniform_k(small, path):
    lib_np, lib = small
    qs = fpsynth.batch_queries(lib_np, 300, 1003).words
    st = check_batch(lib_np, lib, qs, 30, None, path, "uniform k=30")
    assert st["path"] == fps.PATH_NAMES[path]


@pytest.mark.parametrize("path", PATHS)
def test_batch_paths_uneven_k_masks(small, path):
    lib_np, lib = small
    nq = 333
    qs = fpsynth.batch_queries(lib_np, nq, 1004).words
    k, masks = fpsynth.uneven_params(nq, 1004)
    check_batch(lib_np, lib, qs, k, masks, path, "uneven k and masks")


@pytest.mark.parametrize("path,variant", [(fps.PATH_MFMA_I8, v) for v in range(5)] +
                         [(fps.PATH_MFMA_F4, v) for v in range(5)])
def test_mfma_variants(small, path, variant):
    """Every matrix-core tile shape gives the oracle's answer (partial query
    blocks included: 600 queries over 3 masks)."""
    lib_np, lib = small
    nq = 600
    qs = fpsynth.batch_queries(lib_np, nq, 40 + variant).words
    k, masks = fpsynth.uneven_params(nq, 41)
    lib.set_variant(variant)
    try:
        check_batch(lib_np, lib, qs, k, masks, path, f"variant {variant}")
        lib.set_tuning(sample_records=2048, phase_records=10_000)
        check_batch(lib_np, lib, qs, k, masks, path, f"variant {variant} 2-phase")
    finally:
        lib.set_tuning()
        lib.set_variant(-1)


@pytest.mark.parametrize("path", PATHS)
def test_graph_replay(small, path):
    """A launch shape seen again is captured into a HIP graph and replayed with
    new queries; every replay is checked against the oracle, with eager calls
    of other shapes and synchronizations in between."""
    lib_np, lib = small
    nq = 200
    k, masks = fpsynth.uneven_params(nq, 50)
    lib.set_path(path)
    used = []
    try:
        for rep in range(6):
            qs = fpsynth.batch_queries(lib_np, nq, 600 + rep).words
            say("case: graph replay", path, rep)
            hits, off = lib.search_batch(qs, k, masks)
            used.append(lib.last_stats()["graph"])
            ohits, ooff = oracle.search_batch(lib_np.words, qs, k, lib.strides, masks)
            assert np.array_equal(off, ooff) and np.array_equal(hits, ohits), rep
            torch.cuda.synchronize()
            one = lib.search(qs[1], 7, mask=3)
            assert np.array_equal(one, oracle.search(lib_np.words, qs[1], 7,
                                                     ranges=[(0, 75_000)])), rep
    finally:
        lib.set_path(fps.PATH_AUTO)
    if path == fps.PATH_SINGLE:
        assert not any(used), used  # the single-query scan launches directly
    else:
        assert used[0] is False and all(used[1:]), used
    lib.set_graphs(False)
    qs = fpsynth.batch_queries(lib_np, nq, 700).words
    lib.set_path(path)
    hits, off = lib.search_batch(qs, k, masks)
    lib.set_path(fps.PATH_AUTO)
    lib.set_graphs(True)
    assert lib.last_stats()["graph"] is False
    ohits, ooff = oracle.search_batch(lib_np.words, qs, k, lib.strides, masks)
    assert np.array_equal(hits, ohits)


@pytest.mark.parametrize("path", PATHS)
def test_timing_modes(small, path):
    """Device timing is opt-in: results are identical with and without it; with
    it, every call reports positive scan and total device time, also from a
    replayed graph; without it both are zero."""
    lib_np, lib = small
    qs = fpsynth.batch_queries(lib_np, 40, 800).words
    k, masks = fpsynth.uneven_params(40, 800)
    lib.set_path(path)
    try:
        for timing in (False, True, False, True):
            lib.set_timing(timing)
            for rep in range(3):  # eager, eager (seen), graph replay
                say("case: timing", timing, "path", path, "rep", rep)
                hits, off = lib.search_batch(qs, k, masks)
                st = lib.last_stats()
                ohits, ooff = oracle.search_batch(lib_np.words, qs, k, lib.strides, masks)
                assert np.array_equal(off, ooff) and np.array_equal(hits, ohits)
                assert st["scan_launches"] >= 1
                if timing:
                    assert st["scan_ms"] > 0 and st["total_ms"] >= st["scan_ms"], st
                else:
                    assert st["scan_ms"] == 0 and st["total_ms"] == 0, st
            one = lib.search(qs[0], 30)
            st = lib.last_stats()
            assert np.array_equal(one, oracle.search(lib_np.words, qs[0], 30))
            assert (st["scan_ms"] > 0) == timing and (st["total_ms"] > 0) == timing
    finally:
        lib.set_timing(False)
        lib.set_path(fps.PATH_AUTO)


@pytest.mark.parametrize("path", [fps.PATH_SINGLE, fps.PATH_MFMA_F4, fps.PATH_POPCOUNT])
def test_shard_merge(path):
    """The multi-GPU design on one GPU: the library cut into 8 equal strides
    (one per GPU), every query searched on each shard alone with global indices
    (one batch: query i on shard s), the 8 top-k lists merged by (distance,
    index): equal to the search over the whole library and to the oracle."""
    n, G, k = 80_007, 8, 30
    lib_np = fpsynth.make_library(n, 21)
    cuts = [n * s // G for s in range(G + 1)]
    lib = fps.Library(lib_np.words, strides=cuts)
    qs = fpsynth.batch_queries(lib_np, 16, 22).words
    rows = np.repeat(qs, G, axis=0)
    masks = np.tile(np.array([1 << s for s in range(G)], dtype=np.uint32), len(qs))
    lib.set_path(path)
    try:
        say("case: shard merge", path)
        hits, off = lib.search_batch(rows, k, masks)
    finally:
        lib.set_path(fps.PATH_AUTO)
    for i in range(len(qs)):
        parts = []
        for s in range(G):
            h = hits[int(off[i * G + s]):int(off[i * G + s + 1])]
            assert np.all((h["index"] >= cuts[s]) & (h["index"] < cuts[s + 1]))
            parts.append(h)
        allh = np.concatenate(parts)
        merged = allh[np.lexsort((allh["index"], allh["distance"]))][:k]
        whole = lib.search(qs[i], k)
        assert np.array_equal(merged, whole), i
        assert np.array_equal(whole, oracle.search(lib_np.words, qs[i], k)), i


def test_autotuner_and_cache(tmp_path, monkeypatch):
    """AUTO times every candidate on the first batch of a shape, caches the
    winner (also in the FPS_TUNE_CACHE file), and a new handle reuses it."""
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("FPS_TUNE_CACHE", str(cache))
    lib_np = fpsynth.make_library(50_000, 3)
    lib = fps.Library(lib_np.words)
    qs = fpsynth.batch_queries(lib_np, 100, 7).words
    hits, off = lib.search_batch(qs, 30)
    ohits, ooff = oracle.search_batch(lib_np.words, qs, 30)
    assert np.array_equal(off, ooff) and np.array_equal(hits, ohits)
    st = lib.last_stats()
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and '"path"' in lines[0]
    lib2 = fps.Library(lib_np.words)
    hits2, off2 = lib2.search_batch(qs, 30)
    assert np.array_equal(hits2, hits)
    assert len(cache.read_text().splitlines()) == 1  # cached: no second tuning
    st2 = lib2.last_stats()
    assert (st2["path"], st2["variant"]) == (st["path"], st["variant"])


@pytest.fixture(scope="module")
def wide_batch():
    """12,000 queries over a ragged 6,000-record library with three strides: k
    from {0, 1, 7, 30, 5,999, 6,000, 7,000} (0, and k at or beyond the records
    of the query's strides, included) and every stride mask; the oracle's
    answer is computed once."""
    lib_np = fpsynth.make_library(6_000, 21)
    strides = [0, 1_500, 4_100, 6_000]
    lib = fps.Library(lib_np.words, strides=strides)
    nq = 12_000
    qs = fpsynth.batch_queries(lib_np, nq, 22).words
    rng = np.random.default_rng(23)
    k = rng.choice(np.array([0, 1, 7, 30, 5_999, 6_000, 7_000], dtype=np.uint32), nq,
                   p=[0.05, 0.2, 0.3, 0.3, 0.05, 0.05, 0.05]).astype(np.uint32)
    masks = rng.integers(1, 8, nq).astype(np.uint32)
    want = oracle.search_batch(lib_np.words, qs, k, strides, masks)
    return lib_np, lib, qs, k, masks, want


@pytest.mark.parametrize("path", PATHS + [fps.PATH_AUTO])
def test_wide_batch(wide_batch, path):
    """More queries than any benchmark batch, every path against one oracle run."""
    lib_np, lib, qs, k, masks, (ohits, ooff) = wide_batch
    lib.set_path(path)
    say("case: wide batch path", path, "q", len(qs))
    try:
        hits, off = lib.search_batch(qs, k, masks)
    finally:
        lib.set_path(fps.PATH_AUTO)
    assert np.array_equal(off, ooff)
    assert np.array_equal(hits, ohits)


@pytest.mark.parametrize("case", range(32))
def test_random_combinations(case):
    """Seeded random combinations of the dimensions tested one at a time
    elsewhere: library size (ragged), stride cuts, batch size, per-query k
    (0 to beyond n) and masks, on every path.  The case number names its seed."""
    rng = np.random.default_rng(9000 + case)
    n = int(rng.integers(1, 60_000))
    nstr = int(rng.integers(1, 5))
    cuts = sorted(set(int(c) for c in rng.integers(1, max(n, 2), nstr - 1))) if n > 1 else []
    strides = [0] + [c for c in cuts if 0 < c < n] + [n]
    lib_np = fpsynth.make_library(n, 9100 + case)
    lib = fps.Library(lib_np.words, strides=strides)
    ns = len(strides) - 1
    nq = int(rng.integers(1, 700))
    qs = fpsynth.batch_queries(lib_np, nq, 9200 + case).words
    k = rng.choice(np.array([0, 1, 2, 5, 30, 100, 1000, n, n + 3], dtype=np.int64), nq)
    k = np.minimum(k, 2 ** 31).astype(np.uint32)
    masks = rng.integers(1, 2 ** ns, nq).astype(np.uint32)
    say("case: random", case, "n", n, "strides", strides, "q", nq)
    want, woff = oracle.search_batch(lib_np.words, qs, k, strides, masks)
    for path in PATHS:
        lib.set_path(path)
        try:
            hits, off = lib.search_batch(qs, k, masks)
        finally:
            lib.set_path(fps.PATH_AUTO)
        assert np.array_equal(off, woff), (case, path)
        assert np.array_equal(hits, want), (case, path)


@pytest.mark.parametrize("path", PATHS)
def test_all_masks_and_strides(small, path):
    lib_np, lib = small
    qs = fpsynth.batch_queries(lib_np, 7 * 5, 77).words
    masks = np.repeat(np.arange(1, 8, dtype=np.uint32), 5)
    k = np.tile(np.array([1, 10, 30, 100, 1000], dtype=np.uint32), 7)
    check_batch(lib_np, lib, qs, k, masks, path, "every mask")


@pytest.mark.parametrize("n", [1, 63, 511, 513, 2047, 2049, 4097, 33_333])
@pytest.mark.parametrize("path", PATHS)
def test_ragged_sizes(n, path):
    lib_np = fpsynth.make_library(n, 100 + n)
    lib = fps.Library(lib_np.words)
    qs = fpsynth.batch_queries(lib_np, 70, n).words
    for k in (1, 30, n):
        check_batch(lib_np, lib, qs, k, None, path, f"n={n} k={k}")


@pytest.mark.parametrize("path", PATHS)
def test_odd_stride_boundaries(path):
    n = 20_011
    lib_np = fpsynth.make_library(n, 5)
    strides = [0, 1, 2, 515, 1027, 1027, 9_999, 20_010, n]
    lib = fps.Library(lib_np.words, strides=strides)
    nq = 96
    qs = fpsynth.batch_queries(lib_np, nq, 9).words
    rng = np.random.default_rng(3)
    masks = rng.integers(1, 256, size=nq).astype(np.uint32)
    k = rng.choice(np.array([1, 3, 30, 500], dtype=np.uint32), size=nq)
    check_batch(lib_np, lib, qs, k, masks, path, "odd strides")


@pytest.mark.parametrize("path", PATHS)
def test_forced_fallback(small, path):
    lib_np, lib = small
    qs = fpsynth.batch_queries(lib_np, 40, 5).words
    k, masks = fpsynth.uneven_params(40, 6)
    lib.set_tuning(force_fallback=True)
    try:
        st = check_batch(lib_np, lib, qs, k, masks, path, "forced fallback")
        assert st["fallbacks"] == 40
    finally:
        lib.set_tuning()


@pytest.mark.parametrize("sample,phase", [(1024, 2048), (1024, 20_000), (5000, 33_333),
                                          (64, 512), (100_000, 4096)])
@pytest.mark.parametrize("path", PATHS)
def test_two_phase_bounds(small, path, sample, phase):
    """Small bound samples and short first phases: the refined bound path."""
    lib_np, lib = small
    nq = 150
    qs = fpsynth.batch_queries(lib_np, nq, 31).words
    k, masks = fpsynth.uneven_params(nq, 32)
    lib.set_tuning(sample_records=sample, phase_records=phase)
    try:
        check_batch(lib_np, lib, qs, k, masks, path, f"sample {sample} phase {phase}")
        got = lib.search(qs[0], 30)
        assert np.array_equal(got, oracle.search(lib_np.words, qs[0], 30))
    finally:
        lib.set_tuning()


@pytest.mark.parametrize("sample,k,phases", [(4096, 30, 1), (512, 30, 1), (256, 30, 2),
                                             (4096, 500, 2), (64, 1, 1), (64, 100, 2)])
@pytest.mark.parametrize("path", PATHS)
def test_phase_schedule(small, path, sample, k, phases):
    """One scan phase when the first bound admits few records (k * n / sample
    <= 8192), geometric phases otherwise; a batch of 8 and a single query, both
    against the oracle."""
    lib_np, lib = small
    qs = fpsynth.batch_queries(lib_np, 8, 77 + k).words
    lib.set_tuning(sample_records=sample)
    try:
        st = check_batch(lib_np, lib, qs, k, None, path, f"schedule s={sample} k={k}")
        per_phase = 8 if path == fps.PATH_SINGLE else 1
        assert st["scan_launches"] == phases * per_phase, st
        got = lib.search(qs[0], k)
        assert np.array_equal(got, oracle.search(lib_np.words, qs[0], k))
        assert lib.last_stats()["scan_launches"] == phases
    finally:
        lib.set_tuning()


@pytest.mark.parametrize("path", PATHS)
def test_overflow_fallback(small, path):
    lib_np, lib = small
    qs = fpsynth.batch_queries(lib_np, 70, 8).words
    lib.set_tuning(candidate_scale=1e-6, sample_records=1024, phase_records=4096)
    try:
        st = check_batch(lib_np, lib, qs, 30, None, path, "overflow")
        assert st["fallbacks"] > 0
    finally:
        lib.set_tuning()


@pytest.mark.parametrize("path", PATHS)
def test_identical_rows(path):
    """100,000 identical rows: every record ties; k = 1 must return index 0."""
    rec = fpsynth.make_library(1, 51).words[0]
    words = np.tile(rec, (100_000, 1))
    lib = fps.Library(words, strides=[0, 50_000, 100_000])
    qs = np.stack([rec] * 70)
    qs[1::2, 1] ^= np.uint64(1 << 5)
    k = np.array([1, 30, 9000, 20_000, 100_000] * 14, dtype=np.uint32)
    masks = np.array([1, 2, 3] * 24, dtype=np.uint32)[:70]
    check_batch(words_lib(words), lib, qs, k, masks, path, "identical rows")


@pytest.mark.parametrize("k,ties,fallback", [(1, 500, 0), (30, 1000, 0), (5, 1025, 0),
                                              (40, 3000, 0), (30, 8192, None), (7, 8193, 1),
                                              (2000, 0, 0)])
def test_single_query_select_outcomes(k, ties, fallback):
    """One query whose D_k-th distance is shared by `ties` records (planted
    copies of the query): the select ranks up to 1,024 candidates with
    d <= D_k directly, sorts 1,025..8,192 in LDS and leaves more to the exact
    fallback (8,192 ties may also overflow the candidate buffer; the fallback
    answers that too).  Every outcome equals the oracle's top-k."""
    lib_np = fpsynth.make_library(60_000, 91)
    words = lib_np.words.copy()
    q = fpsynth.batch_queries(lib_np, 1, 92).words[0]
    rng = np.random.default_rng(ties + k)
    if ties:
        words[rng.choice(len(words), ties, replace=False)] = q
    say("case: single select outcome k", k, "ties", ties)
    lib = fps.Library(words, strides=[0, 20_000, 60_000])
    try:
        got = lib.search(q, k)
        assert np.array_equal(got, oracle.search(words, q, k))
        if fallback is not None:
            assert lib.last_stats()["fallbacks"] == fallback
    finally:
        lib.close()


def words_lib(words):
    class W:
        pass
    w = W()
    w.words = words
    return w


def test_determinism(small):
    lib_np, lib = small
    qs = fpsynth.batch_queries(lib_np, 256, 21).words
    k, masks = fpsynth.uneven_params(256, 22)
    outs = []
    for path in PATHS:
        lib.set_path(path)
        for _ in range(4):
            h, off = lib.search_batch(qs, k, masks)
            outs.append(h.tobytes() + off.tobytes())
    lib.set_path(fps.PATH_AUTO)
    assert all(o == outs[0] for o in outs)


def test_errors(small):
    lib_np, lib = small
    q = lib_np.words[5].copy()
    bad = q.copy()
    bad[0] |= np.uint64(1)
    with pytest.raises(fps.FPSError) as e:
        lib.search(bad, 30)
    assert e.value.status == fps.FPS_E_FINGERPRINT
    bad = q.copy()
    bad[2] |= np.uint64(1) << np.uint64(40)
    with pytest.raises(fps.FPSError) as e:
        lib.search_batch(np.stack([q, bad]), 30)
    assert e.value.status == fps.FPS_E_FINGERPRINT and "query 1" in str(e.value)
    with pytest.raises(fps.FPSError) as e:
        lib.search(q, 30, mask=0)
    assert e.value.status == fps.FPS_E_ARG
    with pytest.raises(fps.FPSError) as e:
        lib.search(q, 30, mask=0b1000)
    assert e.value.status == fps.FPS_E_ARG
    # a workspace that is too small
    import ctypes
    c = fps.load_library()
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    out = np.empty(30, dtype=fps.HIT_DTYPE)
    n = ctypes.c_uint32()
    rc = c.fps_search(lib.handle, ctypes.c_void_p(q.ctypes.data), 30, fps.MASK_ALL,
                      ctypes.c_void_p(ws.data_ptr()), 1024, ctypes.c_void_p(out.ctypes.data),
                      ctypes.byref(n), None)
    assert rc == fps.FPS_E_NOMEM
    # the handle still works afterwards
    assert np.array_equal(lib.search(q, 30), oracle.search(lib_np.words, q, 30))


@pytest.mark.parametrize("streams,reserve,cap,deadline_us,max_q,wait_us", [
    (3, 0, True, 10_000, 512, 0),   # deadline cap, every stream always available
    (3, 1, True, 1, 128, 0),        # every request late at once: overload, reserve slot runs
    (2, 0, False, 0, 512, 0),       # no deadlines, no cap
    (1, 0, True, 10_000, 512, 3_000),  # a batch waits up to 3 ms for more requests
])
def test_server_alone_vs_mix(small, streams, reserve, cap, deadline_us, max_q, wait_us):
    """Each request's answer is the same alone, in a mix and from the oracle,
    under every batching policy of the server."""
    lib_np, lib = small
    rng = np.random.default_rng(5)
    reqs = []
    for r in range(40):
        nq = int(rng.integers(1, 65))
        qs = fpsynth.batch_queries(lib_np, nq, 5000 + r).words
        k = int(rng.choice([30, 100, 1000]))
        m = int(rng.choice([1, 3, 7]))
        reqs.append((qs, k, m))
    srv = fps.Server(lib, pool_bytes=512 << 20, max_batch_queries=max_q, n_streams=streams,
                     deadline_cap=cap, reserve_streams=reserve, max_wait_us=wait_us)
    try:
        tickets = [srv.submit(qs, k, m, deadline_us=deadline_us) for qs, k, m in reqs]
        mixed = [srv.wait(t) for t in tickets]
        st = srv.stats()
        assert st["requests"] == 40
        for (qs, k, m), (h, off, rs) in zip(reqs, mixed):
            alone, aoff = lib.search_batch(qs, k, np.full(len(qs), m, dtype=np.uint32))
            want, woff = oracle.search_batch(lib_np.words, qs, k, lib.strides,
                                             np.full(len(qs), m, dtype=np.uint32))
            assert np.array_equal(off, woff) and np.array_equal(h, want)
            assert np.array_equal(aoff, woff) and np.array_equal(alone, want)
        assert max(r[2]["batch_queries"] for r in mixed) > 64  # requests were coalesced
        assert max(r[2]["batch_queries"] for r in mixed) <= max(max_q, 64)
        if deadline_us == 1:
            assert st["deadline_misses"] == 40  # a 1 us budget is always missed
    finally:
        srv.close()


def test_server_k_beyond_records(small):
    """k far beyond the records of a request's strides: the server sizes its
    buffers from min(k, n_eff), so the request is answered like a search."""
    lib_np, lib = small
    qs = fpsynth.batch_queries(lib_np, 3, 77).words
    srv = fps.Server(lib, pool_bytes=256 << 20, max_batch_queries=64, n_streams=1)
    try:
        say("case: server k = 2^31 over stride A")
        t = srv.submit(qs, 1 << 31, 0b001)
        h, off, _ = srv.wait(t)
        want, woff = oracle.search_batch(lib_np.words, qs, 1 << 31, lib.strides,
                                         np.full(3, 0b001, dtype=np.uint32))
        assert int(off[-1]) == 3 * 40_000
        assert np.array_equal(off, woff) and np.array_equal(h, want)
    finally:
        srv.close()


def test_server_wait_checks_buffers_first(small):
    """A too-small output buffer is reported without consuming the ticket; the
    same ticket then delivers the results."""
    import ctypes
    lib_np, lib = small
    qs = fpsynth.batch_queries(lib_np, 4, 78).words
    c = fps.load_library()
    srv = fps.Server(lib, pool_bytes=128 << 20, max_batch_queries=64, n_streams=1)
    try:
        say("case: server wait with small buffers")
        t = srv.submit(qs, 30)
        out = np.empty(4 * 30, dtype=fps.HIT_DTYPE)
        off = np.zeros(5, dtype=np.uint64)
        rc = c.fps_server_wait(srv._h, t, ctypes.c_void_p(out.ctypes.data), 4 * 30 - 1,
                               ctypes.c_void_p(off.ctypes.data), 5, None)
        assert rc == fps.FPS_E_ARG and b"needed" in c.fps_last_error()
        rc = c.fps_server_wait(srv._h, t, ctypes.c_void_p(out.ctypes.data), 4 * 30,
                               ctypes.c_void_p(off.ctypes.data), 4, None)
        assert rc == fps.FPS_E_ARG
        h, o, _ = srv.wait(t)
        want, woff = oracle.search_batch(lib_np.words, qs, 30)
        assert np.array_equal(o, woff) and np.array_equal(h, want)
        rc = c.fps_server_wait(srv._h, t, ctypes.c_void_p(out.ctypes.data), 4 * 30,
                               ctypes.c_void_p(off.ctypes.data), 5, None)
        assert rc == fps.FPS_E_ARG  # consumed
    finally:
        srv.close()


def test_server_latency_from_arrival_and_pretuning(small):
    """Latency and deadlines run from the arrival the caller states; shapes
    named at creation are tuned there, others take the default kernel and are
    counted, and both are exact."""
    lib_np, _ = small
    lib = fps.Library(lib_np.words, strides=[0, 40_000, 75_000, 100_000])  # nothing tuned yet
    qs = fpsynth.batch_queries(lib_np, 40, 79).words
    srv = fps.Server(lib, pool_bytes=256 << 20, max_batch_queries=64, n_streams=1,
                     tune_k=[30])
    try:
        say("case: server arrival stamps and pretuning")
        st0 = srv.stats()
        assert st0["untuned_batches"] == 0
        arrival = fps.clock_ns() - 20_000_000  # arrived 20 ms ago
        t = srv.submit(qs[:8], 30, deadline_us=10_000, arrival_ns=arrival)
        h, off, rs = srv.wait(t)
        assert rs["arrival_ns"] == arrival and rs["done_ns"] - arrival >= 20_000_000
        want, woff = oracle.search_batch(lib_np.words, qs[:8], 30)
        assert np.array_equal(h, want)
        st = srv.stats()
        assert st["deadline_misses"] == 1 and st["p50_us"] >= 20_000
        assert st["untuned_batches"] == 0
        t = srv.submit(qs, 999, mask=0b011)  # a shape nobody tuned
        h, off, _ = srv.wait(t)
        want, woff = oracle.search_batch(lib_np.words, qs, 999, lib.strides,
                                         np.full(40, 0b011, dtype=np.uint32))
        assert np.array_equal(off, woff) and np.array_equal(h, want)
        assert srv.stats()["untuned_batches"] == 1
    finally:
        srv.close()
        lib.close()
