"""CPU ORACLE -- test infrastructure, not part of the product.

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of `bench.py`
may import this package.  It shares no code with the GPU path (no kernels,
headers, helpers or tables); both sides only take inputs from `fpsynth`.

The arithmetic lives in `oracle.c` (plain C, no intrinsics): the Manhattan
distance of Section 4.3 evaluated key by key, the top-N of Fig. 3 step 6 with
ties ordered by ascending library index, the stride split of Section 2.1
with the combine-and-sort rule of Section 4.3, and the line-by-line reader of
the library file (Fig. 3 step 1).  This module is argument marshalling around
it, plus the parser of the bracketed query list of Fig. 1 (Fig. 3 step 2),
written here in plain Python.

Every function here is pinned by `tests/test_oracle_pins.py` against
independent facts: brute force with Python integer bit counts and set algebra,
the paper's own broadcast formulation (Section 4.3) written in numpy, library
sorts, planted distances of the generator, the distances printed in Fig. 2
reproduced by a planted library, and metric axioms.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "_oracle.so")

HIT_DTYPE = np.dtype([("index", np.uint32), ("distance", np.uint32)])


def compile_source(src_path: str, so_path: str) -> str:
    tmp = so_path + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread",
                           "-Wall", "-Wextra", "-o", tmp, src_path])
    os.replace(tmp, so_path)
    return so_path


def build(force: bool = True) -> str:
    """Compile oracle.c into _oracle.so (gcc, host code only)."""
    if force or not os.path.exists(_SO):
        compile_source(SOURCE, _SO)
    return _SO


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def _rec(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64).reshape(3))


def mask_ranges(strides, mask) -> list[tuple[int, int]]:
    """Record ranges selected by a stride mask (bit s selects stride s, whose
    records are [strides[s], strides[s+1])).  mask None selects every stride."""
    ns = len(strides) - 1
    sel = range(ns) if mask is None else [s for s in range(ns) if (int(mask) >> s) & 1]
    return [(int(strides[s]), int(strides[s + 1])) for s in sel]


class Oracle:
    """A loaded build of oracle.c."""

    def __init__(self, so_path: str):
        lib = ctypes.CDLL(so_path)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        lib.oracle_distance.argtypes = [vp, vp]
        lib.oracle_distance.restype = u32
        lib.oracle_distances.argtypes = [vp, u64, u64, vp, vp]
        lib.oracle_distances.restype = None
        lib.oracle_search.argtypes = [vp, vp, vp, u32, vp, u64, vp, i32]
        lib.oracle_search.restype = ctypes.c_int64
        lib.oracle_search_batch.argtypes = [vp, vp, vp, vp, u32, vp, u64, vp, vp, vp, i32]
        lib.oracle_search_batch.restype = i32
        lib.oracle_read_text.argtypes = [vp, u64, vp, vp, u64, vp, vp]
        lib.oracle_read_text.restype = ctypes.c_int64
        lib.oracle_distance_w.argtypes = [vp, vp, u32]
        lib.oracle_distance_w.restype = u32
        lib.oracle_distances_w.argtypes = [vp, u32, u64, u64, vp, vp]
        lib.oracle_distances_w.restype = None
        lib.oracle_search_w.argtypes = [vp, u32, vp, vp, u32, vp, u64, vp, i32]
        lib.oracle_search_w.restype = ctypes.c_int64
        self._lib = lib

    def distance(self, a, b) -> int:
        """Section 4.3: sum_{j=1..166} |a_j - b_j| of two packed fingerprints."""
        a, b = _rec(a), _rec(b)
        return int(self._lib.oracle_distance(_p(a), _p(b)))

    def distances(self, lib_words: np.ndarray, query, begin: int = 0,
                  end: int | None = None) -> np.ndarray:
        """Distances of records [begin, end) to the query (uint32)."""
        w = np.ascontiguousarray(lib_words, dtype=np.uint64)
        end = w.shape[0] if end is None else end
        q = _rec(query)
        out = np.empty(end - begin, dtype=np.uint32)
        self._lib.oracle_distances(_p(w), begin, end, _p(q), _p(out))
        return out

    def search(self, lib_words: np.ndarray, query, k: int, ranges=None,
               nthreads: int = 1) -> np.ndarray:
        """Top-k of one query (Fig. 3): structured array of (index, distance) in
        ascending (distance, index) order, min(k, records in range) entries."""
        w = np.ascontiguousarray(lib_words, dtype=np.uint64)
        if ranges is None:
            ranges = [(0, w.shape[0])]
        b = np.array([r[0] for r in ranges], dtype=np.uint64)
        e = np.array([r[1] for r in ranges], dtype=np.uint64)
        total = int((e - b).sum()) if len(ranges) else 0
        want = min(int(k), total)
        out = np.empty(max(want, 1), dtype=HIT_DTYPE)
        q = _rec(query)
        got = self._lib.oracle_search(_p(w), _p(b), _p(e), len(ranges), _p(q), int(k), _p(out),
                                      int(nthreads))
        if got < 0:
            raise MemoryError("oracle_search ran out of memory")
        return out[:got].copy()

    def search_batch(self, lib_words: np.ndarray, queries: np.ndarray, k, strides=None,
                     masks=None, nthreads: int = 1):
        """Independent top-k per query; returns (hits, offsets): query q's hits are
        hits[offsets[q]:offsets[q+1]]."""
        w = np.ascontiguousarray(lib_words, dtype=np.uint64)
        qs = np.ascontiguousarray(queries, dtype=np.uint64).reshape(-1, 3)
        nq = qs.shape[0]
        k = np.broadcast_to(np.asarray(k, dtype=np.uint64), (nq,)).copy()
        strides = [0, w.shape[0]] if strides is None else list(strides)
        ns = len(strides) - 1
        b = np.zeros((nq, ns), dtype=np.uint64)
        e = np.zeros((nq, ns), dtype=np.uint64)
        nr = np.zeros(nq, dtype=np.uint32)
        cap = 0
        for q in range(nq):
            rr = mask_ranges(strides, None if masks is None else masks[q])
            nr[q] = len(rr)
            for r, (lo, hi) in enumerate(rr):
                b[q, r], e[q, r] = lo, hi
            cap += min(int(k[q]), sum(hi - lo for lo, hi in rr))
        out = np.empty(max(cap, 1), dtype=HIT_DTYPE)
        off = np.zeros(nq + 1, dtype=np.uint64)
        rc = self._lib.oracle_search_batch(_p(w), _p(b), _p(e), _p(nr), ns, _p(qs), nq, _p(k),
                                           _p(out), _p(off), int(nthreads))
        if rc != 0:
            raise MemoryError("oracle_search_batch ran out of memory")
        return out[:int(off[-1])].copy(), off

    # -- wider fingerprints (Section 5, remark 3): records of W words, keys 0..64W-1 --
    def distance_w(self, a, b) -> int:
        a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64).reshape(-1))
        b = np.ascontiguousarray(np.asarray(b, dtype=np.uint64).reshape(-1))
        assert a.shape == b.shape
        return int(self._lib.oracle_distance_w(_p(a), _p(b), a.shape[0]))

    def distances_w(self, lib_words: np.ndarray, query, begin: int = 0,
                    end: int | None = None) -> np.ndarray:
        w = np.ascontiguousarray(lib_words, dtype=np.uint64)
        W = w.shape[1]
        end = w.shape[0] if end is None else end
        q = np.ascontiguousarray(np.asarray(query, dtype=np.uint64).reshape(W))
        out = np.empty(end - begin, dtype=np.uint32)
        self._lib.oracle_distances_w(_p(w), W, begin, end, _p(q), _p(out))
        return out

    def search_w(self, lib_words: np.ndarray, query, k: int, ranges=None,
                 nthreads: int = 1) -> np.ndarray:
        """Top-k of one W-word query over (n, W) records, as search()."""
        w = np.ascontiguousarray(lib_words, dtype=np.uint64)
        W = w.shape[1]
        if ranges is None:
            ranges = [(0, w.shape[0])]
        b = np.array([r[0] for r in ranges], dtype=np.uint64)
        e = np.array([r[1] for r in ranges], dtype=np.uint64)
        total = int((e - b).sum()) if len(ranges) else 0
        out = np.empty(max(min(int(k), total), 1), dtype=HIT_DTYPE)
        q = np.ascontiguousarray(np.asarray(query, dtype=np.uint64).reshape(W))
        got = self._lib.oracle_search_w(_p(w), W, _p(b), _p(e), len(ranges), _p(q), int(k),
                                        _p(out), int(nthreads))
        if got < 0:
            raise MemoryError("oracle_search_w ran out of memory")
        return out[:got].copy()

    def search_batch_w(self, lib_words, queries, k, strides=None, masks=None, nthreads: int = 1):
        """Independent top-k per W-word query: (hits, offsets) as search_batch()."""
        w = np.ascontiguousarray(lib_words, dtype=np.uint64)
        qs = np.ascontiguousarray(queries, dtype=np.uint64).reshape(-1, w.shape[1])
        nq = qs.shape[0]
        k = np.broadcast_to(np.asarray(k, dtype=np.int64), (nq,))
        strides = [0, w.shape[0]] if strides is None else list(strides)
        parts, off = [], [0]
        for q in range(nq):
            rr = mask_ranges(strides, None if masks is None else masks[q])
            h = self.search_w(w, qs[q], int(k[q]), rr, nthreads)
            parts.append(h)
            off.append(off[-1] + len(h))
        hits = np.concatenate(parts) if parts else np.empty(0, dtype=HIT_DTYPE)
        return hits, np.array(off, dtype=np.uint64)

    def read_text(self, text):
        """Records of a library file (Fig. 3 step 1): (words (n, 3) uint64,
        ids (n,) uint64).  Raises TextError(line, kind) on the first malformed
        line (kinds in TEXT_ERRORS)."""
        buf = _text_bytes(text)
        cap = int(np.count_nonzero(buf == 10)) + 1
        words = np.zeros((cap, 3), dtype=np.uint64)
        ids = np.zeros(cap, dtype=np.uint64)
        line = ctypes.c_uint64()
        kind = ctypes.c_int()
        got = self._lib.oracle_read_text(_p(buf), len(buf), _p(words), _p(ids), cap,
                                         ctypes.byref(line), ctypes.byref(kind))
        if got < 0:
            raise TextError(int(line.value), int(kind.value))
        return words[:got].copy(), ids[:got].copy()


# Problems of a library-file line, in the order they are checked (oracle.c).
TEXT_ERRORS = {1: "line too long", 2: "id missing or longer than 19 digits",
               3: "no separator after the id", 4: "keys not 166 or 167 characters 0/1",
               5: "position 0 set", 6: "characters after the keys"}


class TextError(ValueError):
    def __init__(self, line: int, kind: int):
        super().__init__(f"line {line}: {TEXT_ERRORS.get(kind, kind)}")
        self.line = line
        self.kind = kind


def _text_bytes(text) -> np.ndarray:
    if isinstance(text, str):
        text = text.encode()
    if isinstance(text, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(text), dtype=np.uint8)
    return np.ascontiguousarray(text, dtype=np.uint8).reshape(-1)


def parse_query(s: str) -> np.ndarray:
    """The target fingerprint as typed into the search box of Fig. 1 (Fig. 3
    step 2): a bracketed, comma-separated list of 0/1 values, blanks allowed
    around every token and one comma allowed before the closing bracket.  166
    values are keys 1..166; 167 values are positions 0..166, of which position
    0 holds no key and must be 0.  Returns the three words (key j at bit j & 63
    of word j >> 6).  Raises ValueError naming the character position."""
    i, n = 0, len(s)

    def skip(i):
        while i < n and s[i] in " \t\r\n":
            i += 1
        return i

    i = skip(i)
    if i >= n or s[i] != "[":
        raise ValueError(f"position {i}: expected '['")
    i += 1
    vals = []
    while True:
        i = skip(i)
        if i < n and s[i] == "]":
            break
        if i < n and s[i] in "01":
            vals.append(int(s[i]))
            i += 1
        else:
            raise ValueError(f"position {i}: expected 0 or 1")
        i = skip(i)
        if i < n and s[i] == ",":
            i += 1
        elif i < n and s[i] == "]":
            break
        else:
            raise ValueError(f"position {i}: expected ',' or ']'")
    i = skip(i + 1)
    if i != n:
        raise ValueError(f"position {i}: characters after ']'")
    if len(vals) not in (166, 167):
        raise ValueError(f"{len(vals)} values; 166 or 167 expected")
    first = 1 if len(vals) == 166 else 0
    if first == 0 and vals[0] != 0:
        raise ValueError("position 0 holds no key and must be 0")
    v = 0
    for c, x in enumerate(vals):
        if x:
            v |= 1 << (first + c)
    return np.array([(v >> (64 * w)) & ((1 << 64) - 1) for w in range(3)], dtype=np.uint64)


def parse_queries(text: str) -> np.ndarray:
    """One bracketed list per line (blank lines skipped): (q, 3) words.  Raises
    ValueError naming the 1-based line."""
    out = []
    for no, line in enumerate(text.split("\n"), start=1):
        if not line.strip():
            continue
        try:
            out.append(parse_query(line))
        except ValueError as e:
            raise ValueError(f"line {no}: {e}") from None
    return np.array(out, dtype=np.uint64).reshape(-1, 3)


_default: Oracle | None = None


def default() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(_SO):
            build(force=True)
        _default = Oracle(_SO)
    return _default


def distance(a, b) -> int:
    return default().distance(a, b)


def distances(lib_words, query, begin: int = 0, end: int | None = None) -> np.ndarray:
    return default().distances(lib_words, query, begin, end)


def search(lib_words, query, k: int, ranges=None, nthreads: int = 1) -> np.ndarray:
    return default().search(lib_words, query, k, ranges, nthreads)


def search_batch(lib_words, queries, k, strides=None, masks=None, nthreads: int = 1):
    return default().search_batch(lib_words, queries, k, strides, masks, nthreads)


def read_text(text):
    return default().read_text(text)


def distance_w(a, b) -> int:
    return default().distance_w(a, b)


def distances_w(lib_words, query, begin: int = 0, end: int | None = None) -> np.ndarray:
    return default().distances_w(lib_words, query, begin, end)


def search_w(lib_words, query, k: int, ranges=None, nthreads: int = 1) -> np.ndarray:
    return default().search_w(lib_words, query, k, ranges, nthreads)


def search_batch_w(lib_words, queries, k, strides=None, masks=None, nthreads: int = 1):
    return default().search_batch_w(lib_words, queries, k, strides, masks, nthreads)
