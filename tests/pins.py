"""Pins of the CPU oracle: facts fixed by the paper and by mathematics, written
independently of the oracle's own code.

Each pin takes an `Oracle` (a loaded build of oracle/oracle.c) and raises
AssertionError if the oracle disagrees.  `tests/test_oracle_pins.py` runs them on
the real oracle; `tests/test_oracle_mutations.py` runs them on builds of the
oracle with planted mistakes and requires that some pin fails for each.

The independent formulations used here:
  * set algebra: for 0/1 keys, sum_j |a_j - b_j| is the size of the symmetric
    difference of the two key sets (Python sets);
  * Python integer bit counts: popcount(a XOR b) and |a| + |b| - 2|a AND b|;
  * the paper's own broadcast (Section 4.3: C_ij = A_ij - b_j, K = row sums of
    |C|) written in numpy on unpacked bits;
  * library sorting (numpy lexsort on (distance, index)) for Fig. 3 step 6;
  * generator planted distances: a copy with F distinct flipped keys is at
    distance F from its source;
  * the distance column printed in Fig. 2, reproduced by a planted library.
"""
from __future__ import annotations

import os
import random

import numpy as np

import fpsynth

KEYS = range(1, 167)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---------------- test-side packing (independent of the oracle) ----------------
def pack(keys) -> np.ndarray:
    v = 0
    for j in keys:
        assert 1 <= j <= 166
        v |= 1 << j
    return np.array([(v >> (64 * w)) & ((1 << 64) - 1) for w in range(3)], dtype=np.uint64)


def as_int(rec) -> int:
    r = [int(x) for x in np.asarray(rec, dtype=np.uint64).reshape(3)]
    return r[0] | (r[1] << 64) | (r[2] << 128)


def key_set(rec) -> set:
    v = as_int(rec)
    return {j for j in KEYS if (v >> j) & 1}


def unpack_matrix(words: np.ndarray) -> np.ndarray:
    """n x 166 int16 matrix of key values, column j-1 = key j."""
    w = np.ascontiguousarray(words, dtype=np.uint64).reshape(-1, 3)
    bits = np.unpackbits(w.view(np.uint8), axis=1, bitorder="little")  # n x 192, bit i of record
    return bits[:, 1:167].astype(np.int16)


def paper_broadcast(words: np.ndarray, query) -> np.ndarray:
    """Section 4.3 / Fig. 3 steps 3-4 in numpy: C = A - b (broadcast), K = SUM(ABS(C))."""
    A = unpack_matrix(words)
    b = unpack_matrix(np.asarray(query).reshape(1, 3))[0]
    C = A - b
    return np.abs(C).sum(axis=1)


def lexsort_topk(K: np.ndarray, k: int, index_base: int = 0):
    """Fig. 3 steps 5-6 with ties by index: sort (K, index) ascending, take first k."""
    idx = np.arange(len(K), dtype=np.int64) + index_base
    order = np.lexsort((idx, K))[:k]
    return idx[order], K[order]


def assert_hits(hits, idx, dist, what=""):
    assert len(hits) == len(idx), f"{what}: {len(hits)} hits, expected {len(idx)}"
    assert np.array_equal(hits["index"].astype(np.int64), np.asarray(idx, dtype=np.int64)), what
    assert np.array_equal(hits["distance"].astype(np.int64), np.asarray(dist, dtype=np.int64)), what


# ---------------- pins ----------------
def pin_set_algebra(orc):
    rnd = random.Random(11)
    for _ in range(400):
        a = set(rnd.sample(list(KEYS), rnd.randint(0, 166)))
        b = set(rnd.sample(list(KEYS), rnd.randint(0, 166)))
        assert orc.distance(pack(a), pack(b)) == len(a ^ b)


def pin_special_cases(orc):
    empty, full = pack([]), pack(KEYS)
    assert orc.distance(empty, full) == 166
    assert orc.distance(full, empty) == 166
    assert orc.distance(full, full) == 0
    for j in KEYS:  # every key counts exactly once, from either side
        assert orc.distance(pack([j]), empty) == 1, j
        assert orc.distance(empty, pack([j])) == 1, j
        assert orc.distance(pack([j]), full) == 165, j


def pin_bitcount_identities(orc):
    lib = fpsynth.make_library(3000, 5)
    rnd = random.Random(3)
    for _ in range(2000):
        a = lib.words[rnd.randrange(lib.n)]
        b = lib.words[rnd.randrange(lib.n)]
        ia, ib = as_int(a), as_int(b)
        d = orc.distance(a, b)
        assert d == (ia ^ ib).bit_count()
        assert d == ia.bit_count() + ib.bit_count() - 2 * (ia & ib).bit_count()


def pin_metric_axioms(orc):
    lib = fpsynth.make_library(2000, 6)
    rnd = random.Random(4)
    for _ in range(1500):
        x, y, z = (lib.words[rnd.randrange(lib.n)] for _ in range(3))
        dxy, dyx = orc.distance(x, y), orc.distance(y, x)
        assert orc.distance(x, x) == 0
        assert dxy == dyx
        assert orc.distance(x, z) <= dxy + orc.distance(y, z)
        assert 0 <= dxy <= 166


def pin_paper_broadcast_distances(orc):
    for seed in (1, 2, 3):
        lib = fpsynth.make_library(10_000, seed)
        q = fpsynth.make_queries(lib, 2, seed + 1000, flips=(0, 6)).words
        for qi in range(2):
            K = paper_broadcast(lib.words, q[qi])
            assert np.array_equal(orc.distances(lib.words, q[qi]).astype(np.int64), K)


def pin_paper_broadcast_topk(orc):
    for seed in (1, 2):
        n = 10_000
        lib = fpsynth.make_library(n, seed)
        q = fpsynth.batch_queries(lib, 4, seed + 2000).words
        for qi in range(4):
            K = paper_broadcast(lib.words, q[qi])
            for k in (1, 2, 30, 1000, n - 1, n, n + 7):
                idx, dist = lexsort_topk(K, k)
                assert_hits(orc.search(lib.words, q[qi], k), idx, dist, f"seed {seed} q {qi} k {k}")


def pin_histogram_invariant(orc):
    lib = fpsynth.make_library(20_000, 9)
    q = fpsynth.batch_queries(lib, 6, 77).words
    for qi in range(6):
        K = paper_broadcast(lib.words, q[qi])
        cum = np.cumsum(np.bincount(K, minlength=167))
        for k in (1, 10, 30, 100, 1000):
            hits = orc.search(lib.words, q[qi], k)
            dk = int(hits["distance"][-1])
            below = int(cum[dk - 1]) if dk > 0 else 0
            assert below < k <= int(cum[dk]), (k, dk)
            assert np.all(np.diff(hits["distance"].astype(np.int64)) >= 0)


def pin_planted_distances(orc):
    lib = fpsynth.make_library(60_000, 12)
    dups = np.nonzero(lib.dup_src >= 0)[0]
    assert len(dups) > 1000
    for i in dups[:3000]:
        assert orc.distance(lib.words[i], lib.words[lib.dup_src[i]]) == lib.dup_flips[i]
    qs = fpsynth.make_queries(lib, 200, 99, flips=(0, 8))
    for q in range(200):
        assert orc.distance(qs.words[q], lib.words[qs.src[q]]) == qs.flips[q]
        top = orc.search(lib.words, qs.words[q], 1)
        assert top["distance"][0] <= qs.flips[q]


def pin_fig2_column(orc):
    """The distances printed in Fig. 2 come back from a library planted to
    contain exactly those near neighbours of the query."""
    printed = []
    with open(os.path.join(GOLDEN, "fig2_top13_distances.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                printed.append(float(line))
    rnd = random.Random(2019)
    qkeys = set(rnd.sample(list(KEYS), 40))
    recs, planted = [], []
    # far records: 30+ keys away from the query (symmetric difference of >= 30)
    for _ in range(5000):
        far = set(qkeys)
        for j in rnd.sample(list(KEYS), 30):
            far ^= {j}
        recs.append(far)
    for d in printed:  # planted neighbours at the printed distances (the first is the query)
        s = set(qkeys)
        for j in rnd.sample(list(KEYS), int(d)):
            s ^= {j}
        planted.append(len(recs))
        recs.insert(rnd.randrange(len(recs) + 1), s)
    words = np.stack([pack(s) for s in recs])
    hits = orc.search(words, pack(qkeys), len(printed))
    assert [float(x) for x in hits["distance"]] == printed
    assert set(hits["distance"].tolist()) <= set(range(167))


def pin_chunked_equals_serial(orc):
    # heavy ties: records drawn from 40 patterns
    base = fpsynth.make_library(40, 21).words
    rnd = np.random.default_rng(5)
    words = base[rnd.integers(0, 40, size=50_000)]
    q = base[3]
    for k in (1, 7, 30, 1000, 20_000, 60_000):
        a = orc.search(words, q, k, nthreads=1)
        b = orc.search(words, q, k, nthreads=8)
        assert np.array_equal(a, b), k
        K = paper_broadcast(words, q)
        idx, dist = lexsort_topk(K, k)
        assert_hits(a, idx, dist, f"ties k {k}")


def pin_strides_merge(orc):
    n = 30_000
    lib = fpsynth.make_library(n, 31)
    strides = [0, 12_000, 21_000, n]
    q = fpsynth.batch_queries(lib, 3, 5).words
    K_all = [paper_broadcast(lib.words, q[i]) for i in range(3)]
    for qi in range(3):
        for mask in range(1, 8):
            rr = [(strides[s], strides[s + 1]) for s in range(3) if (mask >> s) & 1]
            for k in (1, 30, 500):
                # per-stride top-k, combined and sorted (Section 4.3)
                parts = []
                for lo, hi in rr:
                    idx, dist = lexsort_topk(K_all[qi][lo:hi], k, index_base=lo)
                    parts += list(zip(dist.tolist(), idx.tolist()))
                parts.sort()
                parts = parts[:k]
                for nt in (1, 4):
                    hits = orc.search(lib.words, q[qi], k, ranges=rr, nthreads=nt)
                    assert_hits(hits, [p[1] for p in parts], [p[0] for p in parts],
                                f"mask {mask} k {k} nt {nt}")


def pin_k_edges(orc):
    lib = fpsynth.make_library(500, 41)
    q = lib.words[17]
    assert len(orc.search(lib.words, q, 0)) == 0
    assert len(orc.search(lib.words, q, 10, ranges=[])) == 0
    assert len(orc.search(lib.words, q, 10, ranges=[(100, 100)])) == 0
    h = orc.search(lib.words, q, 10_000)
    assert len(h) == 500
    K = paper_broadcast(lib.words, q)
    idx, dist = lexsort_topk(K, 500)
    assert_hits(h, idx, dist, "k > n")
    assert h["index"][0] == 17 or h["distance"][0] == 0


def pin_identical_rows(orc):
    rec = fpsynth.make_library(1, 51).words[0]
    words = np.tile(rec, (10_000, 1))
    q = pack(key_set(rec) ^ {5, 77})
    h = orc.search(words, q, 1)
    assert h["index"][0] == 0 and h["distance"][0] == 2
    h = orc.search(words, q, 30, ranges=[(5000, 10_000)], nthreads=4)
    assert h["index"].tolist() == list(range(5000, 5030))


def pin_batch_equals_single(orc):
    lib = fpsynth.make_library(8000, 61)
    q = fpsynth.batch_queries(lib, 12, 6).words
    k = np.array([1, 10, 30, 100, 1000, 8000, 9000, 0, 5, 30, 30, 2], dtype=np.uint64)
    strides = [0, 3000, 5000, 8000]
    masks = [1, 3, 7, 2, 4, 5, 6, 7, 1, 3, 7, 4]
    hits, off = orc.search_batch(lib.words, q, k, strides, masks)
    for i in range(12):
        rr = [(strides[s], strides[s + 1]) for s in range(3) if (masks[i] >> s) & 1]
        one = orc.search(lib.words, q[i], int(k[i]), ranges=rr)
        assert np.array_equal(hits[int(off[i]):int(off[i + 1])], one), i


# ---------------- the library file and the query box (Fig. 3 steps 1-2, Fig. 1) ----------------
def key_line(ident: str, keys, width: int = 167, sep: str = " ", tail: str = "") -> str:
    """One library-file line written character by character from a key set."""
    first = 0 if width == 167 else 1
    return ident + sep + "".join("1" if j in keys else "0" for j in range(first, 167)) + tail


def pin_text_handwritten(orc):
    rnd = random.Random(17)
    cases = [set(), {1}, {166}, {63, 64}, {127, 128}, {159, 160, 161}, set(KEYS),
             {2, 3, 5, 7, 11, 13, 101, 163}]
    cases += [set(rnd.sample(list(KEYS), rnd.randint(0, 166))) for _ in range(24)]
    idents = ["1", "0007", "9999999999999999999", "11050016", "42"]
    seps = [" ", "\t", ",", "  ", " ,\t"]
    tails = ["", "\r", "  ", "\t\r"]
    lines, want_keys, want_ids = [], [], []
    for i, keys in enumerate(cases):
        ident = idents[i % len(idents)]
        lines.append(key_line(ident, keys, 167 if i % 3 else 166, seps[i % len(seps)],
                              tails[i % len(tails)]))
        want_keys.append(keys)
        want_ids.append(int(ident))
    for final in ("\n", ""):
        words, ids = orc.read_text("\n".join(lines) + final)
        assert len(words) == len(cases)
        for i in range(len(cases)):
            assert key_set(words[i]) == want_keys[i], i
            assert as_int(words[i]) & 1 == 0
            assert int(ids[i]) == want_ids[i], i


def pin_text_errors(orc):
    good = key_line("5", {3, 70})
    bad = {
        1: key_line("5", {3}, tail=" " * 100),
        2: "",
        3: key_line("5", {3}, sep="x"),
        4: key_line("5", {3})[:100] + "2" + key_line("5", {3})[101:],
        5: key_line("5", {0, 3}),
        6: key_line("5", {3}, tail=" #"),
    }
    extra = {2: ["   " + key_line("5", {1}), key_line("1" * 20, {1}), "\r"],
             4: [key_line("5", {1}) + "0", key_line("5", {1}, width=166)[:-1]]}
    for kind, line in bad.items():
        for b in [line] + extra.get(kind, []):
            for at in (1, 4):
                text = "\n".join([good] * (at - 1) + [b] + [good] * 3) + "\n"
                try:
                    orc.read_text(text)
                except ValueError as e:
                    assert (e.line, e.kind) == (at, kind), (kind, at, e.line, e.kind)
                else:
                    raise AssertionError(f"malformed line of kind {kind} accepted")
    # the first malformed line is the one reported
    text = "\n".join([good, bad[6], good, bad[3]])
    try:
        orc.read_text(text)
    except ValueError as e:
        assert (e.line, e.kind) == (2, 6)
    else:
        raise AssertionError("malformed text accepted")
    # a final newline starts no record; the 255-character limit is inclusive
    w, _ = orc.read_text(good + "\n")
    assert len(w) == 1
    w, _ = orc.read_text(key_line("5", {3}, tail=" " * (255 - len(key_line("5", {3})))))
    assert len(w) == 1


def pin_text_roundtrip(orc):
    lib = fpsynth.make_library(20_000, 71)
    ids = fpsynth.make_cids(20_000, 3)
    for width, sep, crlf, final in ((167, " ", False, True), (166, "\t", True, True),
                                    (167, ",", False, False), (166, "  ", True, False)):
        text = fpsynth.library_text(lib.words, ids, width=width, sep=sep, crlf=crlf,
                                    final_eol=final)
        w, i = orc.read_text(text)
        assert np.array_equal(w, lib.words), (width, sep, crlf, final)
        assert np.array_equal(i, ids)


def pin_query_list(orc):
    import oracle
    zeros = "[" + ",".join(["0"] * 166) + ",]"  # the box of Fig. 1, trailing comma
    assert as_int(oracle.parse_query(zeros)) == 0
    rnd = random.Random(23)
    for t in range(40):
        keys = set(rnd.sample(list(KEYS), rnd.randint(0, 166)))
        width = 166 if t % 2 else 167
        first = 0 if width == 167 else 1
        vals = ["1" if j in keys else "0" for j in range(first, 167)]
        sep = [",", ", ", " ,", "\t,\t"][t % 4]
        s = " [" + sep.join(vals) + ("," if t % 3 == 0 else "") + "] "
        assert key_set(oracle.parse_query(s)) == keys, t
    for bad in ("", "[]", "[" + ",".join(["0"] * 165) + "]", "[" + ",".join(["0"] * 168) + "]",
                "[" + ",".join(["0"] * 165 + ["2"]) + "]", "[" + ",".join(["0"] * 166),
                "[" + ",".join(["0"] * 166) + "] x", "[1" + ",0" * 166 + "]",
                "[" + ",,".join(["0"] * 166) + "]", "(" + ",".join(["0"] * 166) + ")"):
        try:
            oracle.parse_query(bad)
        except ValueError:
            continue
        raise AssertionError(f"accepted {bad[:30]!r}")
    many = oracle.parse_queries("\n" + zeros + "\n\n" + zeros.replace("0,]", "1]") + "\n")
    assert many.shape == (2, 3) and key_set(many[1]) == {166}


# ---------------- wider fingerprints (Section 5, remark 3) ----------------
WIDTHS = (2, 16, 32)


def wide_int(rec) -> int:
    return sum(int(x) << (64 * w) for w, x in enumerate(np.asarray(rec, dtype=np.uint64)))


def wide_pack(keys, W) -> np.ndarray:
    v = 0
    for j in keys:
        v |= 1 << j
    return np.array([(v >> (64 * w)) & ((1 << 64) - 1) for w in range(W)], dtype=np.uint64)


def pin_wide_set_algebra(orc):
    rnd = random.Random(31)
    for W in WIDTHS:
        n = 64 * W
        for _ in range(150):
            a = set(rnd.sample(range(n), rnd.randint(0, n)))
            b = set(rnd.sample(range(n), rnd.randint(0, n)))
            assert orc.distance_w(wide_pack(a, W), wide_pack(b, W)) == len(a ^ b), W
        full = wide_pack(range(n), W)
        empty = wide_pack([], W)
        assert orc.distance_w(full, empty) == n
        for j in (0, 1, 63, 64, n - 1):
            assert orc.distance_w(wide_pack([j], W), empty) == 1, (W, j)


def pin_wide_broadcast_topk(orc):
    for W in WIDTHS:
        lib = fpsynth.make_wide_library(6000, W, W)
        qs, _, _ = fpsynth.make_wide_queries(lib, 3, 5)
        A = np.unpackbits(lib.words.view(np.uint8), axis=1, bitorder="little").astype(np.int16)
        for q in qs:
            b = np.unpackbits(q.view(np.uint8), bitorder="little").astype(np.int16)
            K = np.abs(A - b).sum(axis=1)  # Section 4.3: C = A - b, K = SUM(ABS(C))
            assert np.array_equal(orc.distances_w(lib.words, q).astype(np.int64), K), W
            for k in (1, 30, 1000, 6000, 6005):
                idx, dist = lexsort_topk(K, k)
                assert_hits(orc.search_w(lib.words, q, k), idx, dist, f"W {W} k {k}")
                if k in (30, 1000):
                    assert np.array_equal(orc.search_w(lib.words, q, k, nthreads=8),
                                          orc.search_w(lib.words, q, k))


def pin_wide_strides_and_planted(orc):
    W = 16
    lib = fpsynth.make_wide_library(20_000, W, 7)
    strides = [0, 7000, 12000, 20_000]
    qs, src, fl = fpsynth.make_wide_queries(lib, 4, 9, flips=(0, 6), fresh=np.zeros(4))
    for qi in range(4):
        assert orc.distance_w(qs[qi], lib.words[src[qi]]) == fl[qi]
        for mask in (1, 3, 5, 7):
            rr = [(strides[s], strides[s + 1]) for s in range(3) if (mask >> s) & 1]
            parts = []
            for lo, hi in rr:
                d = orc.distances_w(lib.words, qs[qi], lo, hi).astype(np.int64)
                idx, dist = lexsort_topk(d, 30, index_base=lo)
                parts += list(zip(dist.tolist(), idx.tolist()))
            parts.sort()
            h = orc.search_w(lib.words, qs[qi], 30, ranges=rr, nthreads=4)
            assert_hits(h, [p[1] for p in parts[:30]], [p[0] for p in parts[:30]], f"mask {mask}")
    dups = np.nonzero(lib.dup_src >= 0)[0][:500]
    for i in dups:
        assert orc.distance_w(lib.words[i], lib.words[lib.dup_src[i]]) == lib.dup_flips[i]


ALL_PINS = [
    pin_set_algebra, pin_special_cases, pin_bitcount_identities, pin_metric_axioms,
    pin_paper_broadcast_distances, pin_paper_broadcast_topk, pin_histogram_invariant,
    pin_planted_distances, pin_fig2_column, pin_chunked_equals_serial, pin_strides_merge,
    pin_k_edges, pin_identical_rows, pin_batch_equals_single,
    pin_text_handwritten, pin_text_errors, pin_text_roundtrip, pin_query_list,
    pin_wide_set_algebra, pin_wide_broadcast_topk, pin_wide_strides_and_planted,
]
