"""Seeded synthetic MACCS-166-shaped inputs shared by the oracle's tests and the
GPU path's tests and benchmark.

This module draws bits and formats them (the text forms of a library file and of
a typed query): it contains no distance, ranking or parsing arithmetic.
The paper searches the PubChem MACCS-166 library (Sections 4.1-4.2), which is
not available; these generators stand in for it with the library size the
paper reports (95,417,114 records, Section 2.2) and fingerprints of the same
shape: keys 1..166 set with per-key probabilities p_j ~ Beta(0.6, 2.0)
(about a quarter of the keys set), plus 5 % near-duplicate records (copies of
an earlier record with 0-3 distinct keys flipped) so that the zero-distance
and small-distance ties of Fig. 2 and Table 1 occur.

Bit layout: key j (1..166) of a record is bit (j & 63) of 64-bit word j >> 6;
bit 0 and bits 167..191 are zero.  Records are record-major numpy arrays of
shape (n, 3), dtype uint64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

NKEYS = 166
NWORDS = 3
PAPER_N = 95_417_114  # library size of Section 2.2 / Fig. 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_fpsynth.so")
_SRC = os.path.join(_HERE, "gen.c")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c into _fpsynth.so with gcc (host code only)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-shared", "-fPIC", "-pthread",
                               "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        lib = ctypes.CDLL(_SO)
        u64, i32, dbl = ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        vp = ctypes.c_void_p
        lib.fpsynth_library.argtypes = [u64, u64, vp, dbl, i32, i32, vp, vp, vp, i32]
        lib.fpsynth_library.restype = i32
        lib.fpsynth_queries.argtypes = [u64, u64, vp, u64, vp, vp, i32, i32, vp, vp, vp]
        lib.fpsynth_queries.restype = i32
        lib.fpsynth_text_size.argtypes = [vp, u64, i32, u64, i32, i32]
        lib.fpsynth_text_size.restype = u64
        lib.fpsynth_text_write.argtypes = [vp, vp, u64, i32, ctypes.c_char_p, u64, i32, i32,
                                           vp, i32]
        lib.fpsynth_text_write.restype = i32
        lib.fpsynth_wide_library.argtypes = [u64, u64, ctypes.c_uint32, vp, dbl, i32, i32, vp, vp,
                                             vp, i32]
        lib.fpsynth_wide_library.restype = i32
        lib.fpsynth_wide_queries.argtypes = [u64, u64, vp, u64, ctypes.c_uint32, vp, vp, i32, i32,
                                             vp, vp, vp]
        lib.fpsynth_wide_queries.restype = i32
        _lib = lib
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def bit_probabilities(seed: int) -> np.ndarray:
    """p[192]: p_j ~ Beta(0.6, 2.0) for keys j = 1..166, zero elsewhere."""
    rng = np.random.default_rng(seed)
    p = np.zeros(192, dtype=np.float64)
    p[1:NKEYS + 1] = rng.beta(0.6, 2.0, size=NKEYS)
    return p


def thresholds(p: np.ndarray) -> np.ndarray:
    """32-bit thresholds: key j is set when a uniform 32-bit draw is < thr[j]."""
    t = np.floor(np.asarray(p, dtype=np.float64) * 4294967296.0)
    return np.clip(t, 0, 4294967295).astype(np.uint32)


def default_threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(n, 16))


@dataclass
class SynthLibrary:
    words: np.ndarray          # (n, 3) uint64, record-major
    p: np.ndarray              # (192,) per-key set probability
    seed: int
    dup_src: np.ndarray | None = None    # (n,) int32, -1 for fresh records
    dup_flips: np.ndarray | None = None  # (n,) uint8
    strides: list = field(default_factory=list)  # stride begin offsets + end

    @property
    def n(self) -> int:
        return int(self.words.shape[0])


def make_library(n: int, seed: int, dup_frac: float = 0.05, flips=(0, 3),
                 keep_meta: bool = True, nthreads: int | None = None,
                 strides=None) -> SynthLibrary:
    lib = _load()
    p = bit_probabilities(seed)
    thr = thresholds(p)
    words = np.empty((n, NWORDS), dtype=np.uint64)
    src = np.empty(n, dtype=np.int32) if keep_meta else None
    fl = np.empty(n, dtype=np.uint8) if keep_meta else None
    rc = lib.fpsynth_library(seed, n, _ptr(thr), float(dup_frac), int(flips[0]), int(flips[1]),
                             _ptr(words), _ptr(src), _ptr(fl), nthreads or default_threads())
    if rc != 0:
        raise ValueError("fpsynth_library rejected its arguments")
    st = list(strides) if strides is not None else [0, n]
    return SynthLibrary(words=words, p=p, seed=seed, dup_src=src, dup_flips=fl, strides=st)


@dataclass
class SynthQueries:
    words: np.ndarray   # (q, 3) uint64
    src: np.ndarray     # (q,) int64, library record a query was derived from, -1 if fresh
    flips: np.ndarray   # (q,) uint8


def make_queries(lib: SynthLibrary, nq: int, seed: int, flips=(0, 5),
                 fresh=None) -> SynthQueries:
    """nq queries; fresh[q] true draws query q from the per-key model, else it is a
    library record with a uniform number of distinct flips in [flips[0], flips[1]]."""
    c = _load()
    out = np.empty((nq, NWORDS), dtype=np.uint64)
    src = np.empty(nq, dtype=np.int64)
    fl = np.empty(nq, dtype=np.uint8)
    fr = np.zeros(nq, dtype=np.uint8) if fresh is None else np.asarray(fresh, dtype=np.uint8)
    thr = thresholds(lib.p)
    words = np.ascontiguousarray(lib.words)
    rc = c.fpsynth_queries(seed, nq, _ptr(words), lib.n, _ptr(thr), _ptr(fr),
                           int(flips[0]), int(flips[1]), _ptr(out), _ptr(src), _ptr(fl))
    if rc != 0:
        raise ValueError("fpsynth_queries rejected its arguments")
    return SynthQueries(words=out, src=src, flips=fl)


# --------------------------------------------------------------------------
# Workloads.  Sizes follow the paper: a library of 95,417,114 records
# (Section 2.2), top-30 results (Section 2.1, Fig. 2), three strides scanned in
# parallel and merged (Section 2.1, Section 4.3).
# --------------------------------------------------------------------------
PAPER_STRIDES = [0, 40_000_000, 75_000_000, PAPER_N]
K_CHOICES = (1, 10, 30, 100, 1000)
MASK_CHOICES = (0b001, 0b011, 0b111)  # A, A+B, A+B+C


def workload_small(seed: int = 1, n: int = 100_000):
    """100,000 records; one query = a library record with exactly 2 flips; k = 30."""
    lib = make_library(n, seed)
    q = make_queries(lib, 1, seed + 1000, flips=(2, 2))
    return lib, q, [30], None


def workload_paper_single(seed: int = 1, nq: int = 1, qseed: int = 1001, n: int = PAPER_N):
    """95,417,114 records; queries = library records with 0-5 flips; k = 30."""
    lib = make_library(n, seed, keep_meta=False)
    q = make_queries(lib, nq, qseed, flips=(0, 5))
    return lib, q, [30] * nq, None


def batch_queries(lib: SynthLibrary, nq: int, qseed: int) -> SynthQueries:
    """Half library records with 1-8 flips (even q), half fresh draws (odd q)."""
    fresh = (np.arange(nq) % 2).astype(np.uint8)
    return make_queries(lib, nq, qseed, flips=(1, 8), fresh=fresh)


def uneven_params(nq: int, qseed: int):
    """Per-query k uniform over {1, 10, 30, 100, 1000} and stride mask uniform over
    {A, A+B, A+B+C}."""
    rng = np.random.default_rng(qseed)
    k = rng.choice(np.array(K_CHOICES, dtype=np.uint32), size=nq)
    mask = rng.choice(np.array(MASK_CHOICES, dtype=np.uint32), size=nq)
    return k.astype(np.uint32), mask.astype(np.uint32)


def poisson_requests(rate: float, duration_s: float, seed: int, max_q: int = 64,
                     k_choices=(30, 100, 1000)):
    """Request trace for the serving workload: Poisson arrivals at `rate`/s, each
    request with U{1..max_q} queries and one k drawn from k_choices."""
    rng = np.random.default_rng(seed)
    n = max(1, int(rate * duration_s * 1.2) + 16)
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps)
    t = t[t < duration_s]
    nreq = len(t)
    sizes = rng.integers(1, max_q + 1, size=nreq)
    ks = rng.choice(np.array(k_choices, dtype=np.uint32), size=nreq)
    return t, sizes.astype(np.int64), ks.astype(np.uint32)


# --------------------------------------------------------------------------
# Text form of a library (the paper's library file: one line of MACCS text
# and a PubChem CID per molecule; Abstract, Fig. 3 step 1) and of queries (the
# bracketed 0/1 list typed into the search box, Fig. 1).
# --------------------------------------------------------------------------
CID_MODULUS = 2_147_483_647  # 2^31 - 1, a prime


def make_cids(n: int, seed: int) -> np.ndarray:
    """n distinct ids in [1, 2^31 - 1] in an order unrelated to the row order:
    id_i = (a * i + b) mod (2^31 - 1) + 1 with a, b drawn from the seed (a != 0,
    so the map is injective for n < 2^31 - 1)."""
    if n >= CID_MODULUS:
        raise ValueError("too many records for distinct ids")
    rng = np.random.default_rng([seed, 0x636964])
    a = np.uint64(rng.integers(1, CID_MODULUS))
    b = np.uint64(rng.integers(0, CID_MODULUS))
    i = np.arange(n, dtype=np.uint64)
    return (a * i + b) % np.uint64(CID_MODULUS) + np.uint64(1)


def library_text(words: np.ndarray, ids: np.ndarray, width: int = 167, sep: str = " ",
                 crlf: bool = False, final_eol: bool = True,
                 nthreads: int | None = None) -> np.ndarray:
    """Text of a library, one line per record: "<id><sep><keys>" where <keys>
    is 167 characters '0'/'1' for positions 0..166 (width 167; position 0 holds
    no key and is '0') or 166 characters for keys 1..166 (width 166).  Returns
    a uint8 array of the bytes."""
    c = _load()
    w = np.ascontiguousarray(words, dtype=np.uint64).reshape(-1, NWORDS)
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    n = w.shape[0]
    if ids.shape != (n,):
        raise ValueError("one id per record")
    sb = sep.encode()
    size = int(c.fpsynth_text_size(_ptr(ids), n, int(width), len(sb), int(crlf),
                                   int(final_eol)))
    out = np.empty(size, dtype=np.uint8)
    rc = c.fpsynth_text_write(_ptr(w), _ptr(ids), n, int(width), sb, len(sb), int(crlf),
                              int(final_eol), _ptr(out), nthreads or default_threads())
    if rc != 0:
        raise ValueError("fpsynth_text_write rejected its arguments")
    return out


def query_text(words, width: int = 166, trailing_comma: bool = True, spaces: bool = False) -> str:
    """A query as typed into the search box of Fig. 1: "[v,v,...,v,]" with one
    0/1 value per key (keys 1..166 for width 166; positions 0..166 for width
    167)."""
    w = [int(x) for x in np.asarray(words, dtype=np.uint64).reshape(NWORDS)]
    first = 0 if width == 167 else 1
    vals = [str((w[j >> 6] >> (j & 63)) & 1) for j in range(first, NKEYS + 1)]
    s = (", " if spaces else ",").join(vals)
    return "[" + s + ("," if trailing_comma else "") + "]"


# --------------------------------------------------------------------------
# Wider fingerprints (Section 5, concluding remark 3: more features), e.g.
# 1,024 or 2,048 bits: W 64-bit words per record, every bit a key.  Per-bit
# set probabilities p_j ~ Beta(0.3, 8.0) (about 3.6 % of the bits set, the
# sparse shape of hashed circular fingerprints), quantised to multiples of
# 1/256; 5 % near-duplicates with 0-3 distinct flips, as for MACCS.
# --------------------------------------------------------------------------
def wide_thresholds(words: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng([seed, 0x77696465])
    p = rng.beta(0.3, 8.0, size=64 * words)
    return np.clip(np.floor(p * 256.0), 0, 255).astype(np.uint8)


@dataclass
class WideLibrary:
    words: np.ndarray          # (n, W) uint64
    thr8: np.ndarray           # (64 W,) per-bit 8-bit thresholds
    seed: int
    dup_src: np.ndarray | None = None
    dup_flips: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.words.shape[0])

    @property
    def W(self) -> int:
        return int(self.words.shape[1])


def make_wide_library(n: int, words: int, seed: int, dup_frac: float = 0.05, flips=(0, 3),
                      keep_meta: bool = True, nthreads: int | None = None) -> WideLibrary:
    c = _load()
    thr = wide_thresholds(words, seed)
    out = np.empty((n, words), dtype=np.uint64)
    src = np.empty(n, dtype=np.int32) if keep_meta else None
    fl = np.empty(n, dtype=np.uint8) if keep_meta else None
    rc = c.fpsynth_wide_library(seed, n, words, _ptr(thr), float(dup_frac), int(flips[0]),
                                int(flips[1]), _ptr(out), _ptr(src), _ptr(fl),
                                nthreads or default_threads())
    if rc != 0:
        raise ValueError("fpsynth_wide_library rejected its arguments")
    return WideLibrary(words=out, thr8=thr, seed=seed, dup_src=src, dup_flips=fl)


def make_wide_queries(lib: WideLibrary, nq: int, seed: int, flips=(1, 8), fresh=None):
    """Library records with flipped keys (or fresh draws where fresh[q] != 0):
    returns (words (nq, W), src (nq,), flips (nq,))."""
    c = _load()
    W = lib.W
    out = np.empty((nq, W), dtype=np.uint64)
    src = np.empty(nq, dtype=np.int64)
    fl = np.empty(nq, dtype=np.uint8)
    fr = (np.arange(nq) % 2).astype(np.uint8) if fresh is None else np.asarray(fresh, np.uint8)
    words = np.ascontiguousarray(lib.words)
    rc = c.fpsynth_wide_queries(seed, nq, _ptr(words), lib.n, W, _ptr(lib.thr8), _ptr(fr),
                                int(flips[0]), int(flips[1]), _ptr(out), _ptr(src), _ptr(fl))
    if rc != 0:
        raise ValueError("fpsynth_wide_queries rejected its arguments")
    return out, src, fl
