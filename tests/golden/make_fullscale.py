#!/usr/bin/env python3
"""Expected results of the full-size workloads, written by the CPU oracle alone.

This script imports only the input generator (`fpsynth`) and the oracle
(`oracle`): no value in its output comes from the GPU path.  It rebuilds the
library of 95,417,114 records that the full-size tests and the benchmark use
(Section 2.2 gives the size; seed 1), and for every query of their workloads
computes the top-k of Fig. 3 (ascending (distance, index), Section 4.3
distance) with the oracle's threaded chunk-and-merge form:

  single : 32 queries of seed 1001 (library records with 0-5 flips), top-30
           over the whole library -- the benchmark's headline queries;
  batch  : 1,024 queries of seed 1003 (half library records with 1-8 flips,
           half fresh draws), top-1,000 over the whole library; the top-30,
           top-100 and top-1,000 prefixes serve the batch workload and the
           served requests (k in {30, 100, 1000});
  uneven : 4,096 queries of seed 1004 with per-query k over
           {1, 10, 30, 100, 1000} and stride masks over {A, A+B, A+B+C}
           (strides 40,000,000 / 35,000,000 / 20,417,114; Section 2.1).

The top-k for a smaller k is a prefix of the top-k for a larger one, because
the (distance, index) order is total.

Outputs (in this directory unless --out-dir is given):
  fullscale_95M.json : generator parameters, SHA-256 of the library's words and
                       of every query set, the stride table, the hash rule;
  fullscale_95M.npz  : full top-30 arrays for the single and batch queries,
                       16-byte SHA-256 prefixes of every other result list, the
                       result counts and the last distances.

A result list hashes as the SHA-256 of its (uint32 index, uint32 distance)
little-endian pairs in result order, truncated to its first 16 bytes.

oracle.c is compiled here with `gcc -O3 -march=native` (the tests build the
same source with -O2; the arithmetic is integer, so both builds agree, which
the full-size GPU test spot-checks).  At about 0.07 G comparisons/s on 8 host
threads the whole run takes about 1.5 hours.

Usage: python tests/golden/make_fullscale.py [--threads N] [--checkpoint FILE]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fpsynth  # noqa: E402
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_SEED = 1
SINGLE_SEED, SINGLE_NQ, SINGLE_K = 1001, 32, 30
BATCH_SEED, BATCH_NQ, BATCH_K = 1003, 1024, 1000
UNEVEN_SEED, UNEVEN_NQ = 1004, 4096
HASH_BYTES = 16


def hit_hash(h: np.ndarray) -> bytes:
    """First 16 bytes of SHA-256 over (uint32 index, uint32 distance) pairs."""
    a = np.empty((len(h), 2), dtype="<u4")
    a[:, 0] = h["index"]
    a[:, 1] = h["distance"]
    return hashlib.sha256(a.tobytes()).digest()[:HASH_BYTES]


def words_sha(w: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(w, dtype="<u8").tobytes()).hexdigest()


class Checkpoint:
    """Per-query results kept in a file so an interrupted run resumes."""

    def __init__(self, path):
        self.path = path
        self.data = {}
        if path and os.path.exists(path):
            with np.load(path, allow_pickle=False) as z:
                self.data = {k: z[k] for k in z.files}

    def get(self, key):
        return self.data.get(key)

    def put(self, key, value):
        self.data[key] = value

    def save(self):
        if self.path:
            tmp = self.path + ".tmp.npz"
            np.savez(tmp, **self.data)
            os.replace(tmp, self.path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--out-dir", default=HERE)
    ap.add_argument("--checkpoint", default=None)
    args = ap.parse_args()

    so = os.path.join(tempfile.mkdtemp(prefix="oracle_o3_"), "oracle_o3.so")
    subprocess_build(so)
    orc = oracle.Oracle(so)
    ck = Checkpoint(args.checkpoint)
    t0 = time.time()

    def say(*a):
        print(f"[{time.time() - t0:8.1f}s]", *a, flush=True)

    n = fpsynth.PAPER_N
    strides = list(fpsynth.PAPER_STRIDES)
    lib = fpsynth.make_library(n, LIB_SEED, keep_meta=False)
    words = lib.words
    lib_sha = words_sha(words)
    say("library", n, "records, sha256", lib_sha)

    def run(tag, queries, ks, masks, keep_top):
        """Top-k of every query; returns per-query (hits[:keep_top], count, hash of
        each requested prefix)."""
        nq = len(queries)
        done = ck.get(tag + "_done")
        res_hash = ck.get(tag + "_hash")
        if done is None:
            done = np.zeros(nq, dtype=np.uint8)
            res_hash = np.zeros((nq, len(keep_top[1]), HASH_BYTES), dtype=np.uint8)
            top_idx = np.zeros((nq, keep_top[0]), dtype=np.uint32)
            top_d = np.zeros((nq, keep_top[0]), dtype=np.uint8)
            count = np.zeros(nq, dtype=np.uint32)
            last = np.zeros(nq, dtype=np.uint8)
        else:
            top_idx, top_d = ck.get(tag + "_top_idx"), ck.get(tag + "_top_d")
            count, last = ck.get(tag + "_count"), ck.get(tag + "_last")
        tq = time.time()
        ndone0 = int(done.sum())
        for q in range(nq):
            if done[q]:
                continue
            m = None if masks is None else int(masks[q])
            rr = oracle.mask_ranges(strides, m)
            h = orc.search(words, queries[q], int(ks[q]), ranges=rr, nthreads=args.threads)
            count[q] = len(h)
            last[q] = h["distance"][-1] if len(h) else 0
            kt = min(keep_top[0], len(h))
            top_idx[q, :kt] = h["index"][:kt]
            top_d[q, :kt] = h["distance"][:kt]
            for j, kp in enumerate(keep_top[1]):
                res_hash[q, j] = np.frombuffer(hit_hash(h[:kp]), dtype=np.uint8)
            done[q] = 1
            nd = int(done.sum())
            if nd % 16 == 0 or nd == nq:
                rate = (nd - ndone0) / max(1e-9, time.time() - tq)
                say(f"{tag}: {nd}/{nq} queries, eta {(nq - nd) / max(rate, 1e-9) / 60:.1f} min")
                for key, val in ((tag + "_done", done), (tag + "_hash", res_hash),
                                 (tag + "_top_idx", top_idx), (tag + "_top_d", top_d),
                                 (tag + "_count", count), (tag + "_last", last)):
                    ck.put(key, val)
                ck.save()
        return top_idx, top_d, count, last, res_hash

    # single queries of the headline workload
    sq = fpsynth.make_queries(lib, SINGLE_NQ, SINGLE_SEED, flips=(0, 5)).words
    s_idx, s_d, s_cnt, _, s_hash = run("single", sq, [SINGLE_K] * SINGLE_NQ, None,
                                       (SINGLE_K, [SINGLE_K]))
    # the 1,024-query batch at top-1,000 (prefixes for k = 30 and 100)
    bq = fpsynth.batch_queries(lib, BATCH_NQ, BATCH_SEED).words
    b_idx, b_d, b_cnt, b_last, b_hash = run("batch", bq, [BATCH_K] * BATCH_NQ, None,
                                            (30, [30, 100, 1000]))
    # the uneven 4,096-query batch: per-query k and stride mask
    uq = fpsynth.batch_queries(lib, UNEVEN_NQ, UNEVEN_SEED).words
    uk, um = fpsynth.uneven_params(UNEVEN_NQ, UNEVEN_SEED)
    _, _, u_cnt, u_last, u_hash = run("uneven", uq, uk, um, (1, [1 << 30]))

    os.makedirs(args.out_dir, exist_ok=True)
    np.savez_compressed(
        os.path.join(args.out_dir, "fullscale_95M.npz"),
        single_index=s_idx, single_distance=s_d, single_count=s_cnt,
        batch_index=b_idx, batch_distance=b_d, batch_count=b_cnt,
        batch_top30_hash=b_hash[:, 0], batch_top100_hash=b_hash[:, 1],
        batch_top1000_hash=b_hash[:, 2], batch_last1000=b_last,
        uneven_hash=u_hash[:, 0], uneven_count=u_cnt, uneven_last=u_last)
    meta = {
        "what": "CPU-oracle results of the full-size workloads (Fig. 3 top-k, Section 4.3 "
                "distance, ascending (distance, index)); written by tests/golden/make_fullscale.py",
        "library": {"n": n, "seed": LIB_SEED, "generator": "fpsynth.make_library(n, 1)",
                    "words_sha256": lib_sha, "strides": strides},
        "single": {"seed": SINGLE_SEED, "nq": SINGLE_NQ, "k": SINGLE_K, "flips": [0, 5],
                   "queries_sha256": words_sha(sq)},
        "batch": {"seed": BATCH_SEED, "nq": BATCH_NQ, "k_computed": BATCH_K,
                  "prefix_hashes": [30, 100, 1000], "queries_sha256": words_sha(bq)},
        "uneven": {"seed": UNEVEN_SEED, "nq": UNEVEN_NQ, "queries_sha256": words_sha(uq),
                   "k_sha256": hashlib.sha256(uk.astype("<u4").tobytes()).hexdigest(),
                   "mask_sha256": hashlib.sha256(um.astype("<u4").tobytes()).hexdigest()},
        "hash_rule": "first 16 bytes of SHA-256 over the (uint32 index, uint32 distance) "
                     "little-endian pairs of a result list, in result order",
        "oracle_build": "gcc -O3 -march=native -std=c11 of oracle/oracle.c",
        "threads": args.threads,
        "seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(args.out_dir, "fullscale_95M.json"), "w") as f:
        json.dump(meta, f, indent=1)
        f.write("\n")
    say("written to", args.out_dir)


def subprocess_build(so):
    import subprocess
    subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c11", "-shared", "-fPIC",
                           "-pthread", "-o", so, oracle.SOURCE])


if __name__ == "__main__":
    main()
