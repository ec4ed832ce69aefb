#!/usr/bin/env python3
"""Benchmark of the exact MACCS-166 top-k engine on one MI355X.

Headline (value): one query, top-30, against 95,417,114 synthetic MACCS-shaped
fingerprints resident in HBM -- the library size and k of the paper (Section
2.2, Fig. 2) -- in G fingerprint comparisons per second, end to end through
fps_search (query upload, bound, scan, select, result download).  Every step
uses a different query (a library record with 0-5 flipped keys).

Also measured in the same run (secondary objects of the JSON line):
  small   : 100,000 records, one query (a library record with 2 flips), top-30:
            latency in microseconds (the library sits in the GPU's caches)
  shard   : one query on one eighth of the library (one GPU's share of a
            library-sharded search)
  batch   : 1024 queries (half library records with 1-8 flips, half fresh),
            k = 30; a new query set on every repeat
  uneven  : 4096 queries, k uniform over {1,10,30,100,1000}, masks over
            {A, A+B, A+B+C} of strides 40M / 35M / 20.4M; new sets per repeat
  serving : Poisson request arrivals, 1-64 queries per request, k in
            {30,100,1000}, 10 ms deadline.  Every request carries its scheduled
            arrival time, so latency (arrival to results) includes any wait
            for admission; offered, admitted and completed rates side by side
  parity  : the results of the timed full-size queries compared, after the
            timed regions, with expected values the CPU oracle wrote
            (tests/golden/fullscale_95M.*), when those files are present
  cpu_baseline : the CPU oracle on the host's cores, on bounded samples.

Inputs are synthetic (fpsynth): the PubChem library of the paper is not
available.  One JSON line is printed on stdout.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, 8 TB/s
INT8_PEAK_TOPS = 5000.0      # dense int8 MFMA, 5.0 POP/s
FP4_PEAK_TFLOPS = 10100.0    # dense fp4 MFMA, 10.1 PFLOP/s
ALGO_BYTES_PER_RECORD = 166 / 8   # 166 keys = 20.75 bytes of fingerprint
LAYOUT_BYTES_PER_RECORD = 21      # as stored: u64 + u64 + u32 + u8
ALGO_OPS_PER_PAIR = 2 * 166       # one multiply-add per key in the dot form
PAPER_N = 95_417_114
GOLDEN = os.path.join(ROOT, "tests", "golden", "fullscale_95M")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# HBM traffic of the single-query scan kernel, from two rocprofv3 counter runs
# (FETCH_SIZE, WRITE_SIZE) scaled by a calibration copy; valid only while the
# kernel sources hash to what the summary records.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_scan_single.single_top30_95M.hbm_traffic.txt")
TRAFFIC_SOURCES = ["paper_1906_06170_amd/csrc/kernels.hip", "paper_1906_06170_amd/csrc/cand.h",
                   "paper_1906_06170_amd/csrc/fps_internal.h"]


def measured_traffic():
    try:
        lines = open(TRAFFIC_PROFILE).read().splitlines()
    except OSError:
        return None
    vals = dict(l.split(":", 1) for l in lines if l.startswith(("traffic_bytes_per_launch:",
                                                                  "source_sha256:")))
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if vals.get("source_sha256", "").strip() != h.hexdigest():
        return None
    return float(vals["traffic_bytes_per_launch"])


def hit_hash(h: np.ndarray) -> bytes:
    """The goldens' hash rule: first 16 bytes of SHA-256 over the (uint32 index,
    uint32 distance) little-endian pairs of a result list."""
    a = np.empty((len(h), 2), dtype="<u4")
    a[:, 0] = h["index"]
    a[:, 1] = h["distance"]
    return hashlib.sha256(a.tobytes()).digest()[:16]


class Goldens:
    """Expected full-size results written by the oracle (None when absent)."""

    def __init__(self, lib_words):
        self.ok = False
        try:
            self.meta = json.load(open(GOLDEN + ".json"))
            self.z = dict(np.load(GOLDEN + ".npz", allow_pickle=False))
        except OSError:
            return
        digest = hashlib.sha256(np.ascontiguousarray(lib_words, dtype="<u8").tobytes())
        self.ok = digest.hexdigest() == self.meta["library"]["words_sha256"]
        if not self.ok:
            log("goldens do not match this library; parity not checked")

    def single(self, i, h):
        d = self.z["single_distance"][i]
        return (len(h) == 30 and np.array_equal(h["index"], self.z["single_index"][i])
                and np.array_equal(h["distance"], d))

    def batch(self, i, h):
        return hit_hash(h) == bytes(self.z["batch_top30_hash"][i])

    def uneven(self, i, h):
        return hit_hash(h) == bytes(self.z["uneven_hash"][i])


def cpu_ident():
    """Family, model and stepping from /proc/cpuinfo (they name the exact part
    when the model-name string is generic)."""
    vals = {}
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k = k.strip()
            if k in ("vendor_id", "cpu family", "model", "stepping") and k not in vals:
                vals[k] = v.strip()
    except OSError:
        pass
    return vals


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=PAPER_N)
    ap.add_argument("--only", default="all",
                    help="comma list of: small,single,shard,batch,uneven,serve,ingest,cluster,wide,"
                         "cpu")
    ap.add_argument("--wide-n", type=int, default=24_000_000,
                    help="records of the 2,048-key library of the wide leg")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--serve-warmup", type=float, default=1.0,
                    help="seconds of arrivals per rate excluded from the statistics")
    ap.add_argument("--serve-rates", default="200,1000,5000")
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first (counter calibration)")
    ap.add_argument("--path", default="auto", help="batch path: auto|popcount|mfma_i8|mfma_f4")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the engine runs on one GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    legs = set(args.only.split(",")) if args.only != "all" else {
        "small", "single", "shard", "batch", "uneven", "serve", "ingest", "cluster", "wide", "cpu"}

    import torch
    import fpsynth
    import paper_1906_06170_amd as fps

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib << 20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    out = {}
    parity = {}

    # ---------------- 100,000 records (latency) ----------------
    if "small" in legs:
        out["small"] = small_leg(fps, fpsynth, args)

    t0 = time.time()
    n = args.n
    strides = [0, min(40_000_000, n), min(75_000_000, n), n]
    lib_np = fpsynth.make_library(n, 1, keep_meta=False)
    log(f"library: {n} records generated in {time.time() - t0:.1f}s")
    gold = Goldens(lib_np.words) if n == PAPER_N else None
    t1 = time.time()
    lib = fps.Library(lib_np.words, strides=strides)
    log(f"uploaded in {time.time() - t1:.1f}s")

    # ---------------- single query ----------------
    K, W = args.steps, args.warmup
    qs = fpsynth.make_queries(lib_np, K + W, 1001, flips=(0, 5)).words
    single = None
    if "single" in legs:
        for i in range(W):
            lib.search(qs[i], 30)
        torch.cuda.synchronize()
        # the timed steps run untimed on the device (no HIP events) ...
        per_q, got = [], []
        t = time.perf_counter()
        for i in range(W, W + K):
            tq = time.perf_counter()
            got.append(lib.search(qs[i], 30))  # synchronous: the hits are on the host
            per_q.append(time.perf_counter() - tq)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        ms = el * 1000 / K
        per_q = np.array(per_q) * 1000
        # ... then the same queries again with HIP events around every kernel
        # phase: the scan kernel's duration for the roofline
        lib.set_timing(True)
        st0 = lib.last_stats()
        t = time.perf_counter()
        for i in range(W, W + K):
            lib.search(qs[i], 30)
        torch.cuda.synchronize()
        timed_ms = (time.perf_counter() - t) * 1000 / K
        st1 = lib.last_stats()
        lib.set_timing(False)
        scan_ms = st1["scan_ms_sum"] - st0["scan_ms_sum"]          # HIP events, scan launches
        launches = st1["scan_launches_sum"] - st0["scan_launches_sum"]
        dev_ms = (st1["total_ms_sum"] - st0["total_ms_sum"]) / K
        per_query_scan = scan_ms / K
        achieved = ALGO_BYTES_PER_RECORD * n / (per_query_scan * 1e-3) / 1e9
        layout = LAYOUT_BYTES_PER_RECORD * n / (per_query_scan * 1e-3) / 1e9
        single = {
            "ms_per_query": ms, "qps": 1000.0 / ms,
            "ms_per_query_median": float(np.median(per_q)), "ms_per_query_min": float(per_q.min()),
            "ms_per_query_max": float(per_q.max()),
            "gcmp_s": n / (ms * 1e-3) / 1e9,
            "scan_ms_per_query": per_query_scan,
            "scan_launches_per_query": launches / K,
            "scan_launch_avg_ms": scan_ms / max(1, launches),
            "device_ms_avg": dev_ms, "graph_replay": bool(st1["graph"]),
            "ms_per_query_with_timing_events": timed_ms,
            "layout_gbs": layout, "layout_frac": layout / HBM_PEAK_GBS,
            "hbm_frac_end_to_end": ALGO_BYTES_PER_RECORD * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        }
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": measured_traffic(),
                           "kernel": "k_scan_single",
                           "bytes_per_launch": ALGO_BYTES_PER_RECORD * n / max(1, launches / K),
                           "launch_avg_ms": scan_ms / max(1, launches)}
        if gold and gold.ok:
            ok = sum(gold.single(W + j, h) for j, h in enumerate(got) if W + j < 32)
            parity["single"] = f"{ok}/{min(K, 32 - W)} equal to the oracle"
        log("single:", json.dumps(single))

    # ---------------- one GPU's shard of an 8-GPU library ----------------
    # The library cut into 8 equal strides; a query restricted to one of them
    # is the per-GPU share of a library-sharded search (global indices; the
    # eight top-k lists merge by (distance, index)).
    if "shard" in legs:
        G = 8
        cuts = [n * s // G for s in range(G + 1)]
        lib8 = fps.Library(lib_np.words, strides=cuts)
        for i in range(W):
            lib8.search(qs[i], 30, mask=1)
        t = time.perf_counter()
        for i in range(W, W + K):
            lib8.search(qs[i], 30, mask=1)
        sh_ms = (time.perf_counter() - t) * 1000 / K
        lib8.set_timing(True)
        s0 = lib8.last_stats()
        for i in range(W, W + K):
            lib8.search(qs[i], 30, mask=1)
        s1 = lib8.last_stats()
        sh_scan = (s1["scan_ms_sum"] - s0["scan_ms_sum"]) / K
        nsh = cuts[1] - cuts[0]
        out["shard"] = {"shards": G, "shard_records": nsh, "ms_per_query": sh_ms,
                        "gcmp_s": nsh / (sh_ms * 1e-3) / 1e9, "scan_ms_per_query": sh_scan,
                        "scan_hbm_frac": ALGO_BYTES_PER_RECORD * nsh / (sh_scan * 1e-3) / 1e9
                        / HBM_PEAK_GBS}
        lib8.close()
        log("shard:", json.dumps(out["shard"]))

    # ---------------- batch of 1024 ----------------
    path = {"auto": fps.PATH_AUTO, "popcount": fps.PATH_POPCOUNT,
            "mfma_i8": fps.PATH_MFMA_I8, "mfma_f4": fps.PATH_MFMA_F4}[args.path]
    if "batch" in legs:
        lib.set_path(path)
        lib.set_timing(True)  # events cost microseconds against a multi-ms batch
        warm = fpsynth.batch_queries(lib_np, 1024, 999).words
        for _ in range(2):  # first sight: autotuner; second: graph capture
            lib.search_batch(warm, 30)
        torch.cuda.synchronize()
        # a new query set on every repeat; repeat 0 is the set the oracle's
        # expected results cover
        sets = [fpsynth.batch_queries(lib_np, 1024, 1003 + 100 * r).words
                for r in range(args.batch_steps)]
        times, scans, first = [], [], None
        for r in range(args.batch_steps):
            t = time.perf_counter()
            h, o = lib.search_batch(sets[r], 30)
            times.append(time.perf_counter() - t)
            scans.append(lib.last_stats())
            if r == 0:
                first = (h.copy(), o.copy())
        ms = float(np.median(times)) * 1000
        scan = float(np.median([s["scan_ms"] for s in scans]))
        pairs = 1024 * n
        b = {"queries": 1024, "k": 30, "path": scans[-1]["path"], "ms": ms,
             "ms_min": float(np.min(times)) * 1000,
             "qps": 1024 / (ms * 1e-3), "gcmp_s": pairs / (ms * 1e-3) / 1e9,
             "scan_kernel_ms": scan, "candidates": scans[-1]["candidates"],
             "fallbacks": scans[-1]["fallbacks"], "variant": scans[-1]["variant"],
             "graph_replay": scans[-1]["graph"], "query_sets": args.batch_steps}
        if single:
            b["speedup_vs_single_qps"] = b["qps"] / single["qps"]
        if scans[-1]["path"] in ("mfma_i8", "mfma_f4"):
            # Algorithmic operations: one multiply-add per key per pair; each path
            # is priced against the dense peak of its own MFMA data type.
            tops = ALGO_OPS_PER_PAIR * pairs / (scan * 1e-3) / 1e12
            i8 = scans[-1]["path"] == "mfma_i8"
            peak = INT8_PEAK_TOPS if i8 else FP4_PEAK_TFLOPS
            b["roofline"] = {"bound": "mfma", "achieved": tops, "peak": peak,
                             "unit": "TOP/s" if i8 else "TFLOP/s", "frac": tops / peak,
                             "dtype": "i8" if i8 else "fp4"}
        if gold and gold.ok:
            h, o = first
            ok = sum(gold.batch(i, h[int(o[i]):int(o[i + 1])]) for i in range(1024))
            parity["batch"] = f"{ok}/1024 equal to the oracle (query set 0)"
        out["batch"] = b
        lib.set_path(fps.PATH_AUTO)
        lib.set_timing(False)
        log("batch:", json.dumps(b))

    # ---------------- uneven 4096 ----------------
    if "uneven" in legs:
        lib.set_path(path)
        lib.set_timing(True)
        reps = max(2, args.batch_steps // 2)
        sets = []
        for r in range(reps):
            qseed = 1004 + 100 * r
            uk, um = fpsynth.uneven_params(4096, qseed)
            sets.append((fpsynth.batch_queries(lib_np, 4096, qseed).words, uk, um))
        wq, wk, wm = sets[-1]
        for _ in range(2):  # tuner, then graph capture (same shape as every set)
            lib.search_batch(wq, wk, wm)
        times, scans, first = [], [], None
        for r in range(reps):
            t = time.perf_counter()
            h, o = lib.search_batch(*sets[r])
            times.append(time.perf_counter() - t)
            scans.append(lib.last_stats())
            if r == 0:
                first = (h.copy(), o.copy())
        ms = float(np.median(times)) * 1000
        neff = {1: strides[1], 3: strides[2], 7: n}
        pairs = float(np.mean([sum(neff[int(m)] for m in s[2]) for s in sets]))
        u = {"queries": 4096, "path": scans[-1]["path"], "ms": ms,
             "ms_min": float(np.min(times)) * 1000,
             "qps": 4096 / (ms * 1e-3), "gcmp_s": pairs / (ms * 1e-3) / 1e9,
             "scan_kernel_ms": float(np.median([s["scan_ms"] for s in scans])),
             "fallbacks": scans[-1]["fallbacks"], "query_sets": reps}
        if scans[-1]["path"] in ("mfma_i8", "mfma_f4"):
            i8 = scans[-1]["path"] == "mfma_i8"
            tops = ALGO_OPS_PER_PAIR * pairs / (u["scan_kernel_ms"] * 1e-3) / 1e12
            peak = INT8_PEAK_TOPS if i8 else FP4_PEAK_TFLOPS
            u["roofline"] = {"bound": "mfma", "achieved": tops, "peak": peak,
                             "unit": "TOP/s" if i8 else "TFLOP/s", "frac": tops / peak,
                             "dtype": "i8" if i8 else "fp4"}
        if gold and gold.ok:
            h, o = first
            ok = sum(gold.uneven(i, h[int(o[i]):int(o[i + 1])]) for i in range(4096))
            parity["uneven"] = f"{ok}/4096 equal to the oracle (query set 0)"
        out["uneven"] = u
        lib.set_path(fps.PATH_AUTO)
        lib.set_timing(False)
        log("uneven:", json.dumps(u))

    # ---------------- serving ----------------
    if "serve" in legs:
        out["serving"] = serve(lib, lib_np, args, fps, fpsynth)

    # ---------------- wider fingerprints ----------------
    if "wide" in legs:
        out["wide"] = wide_leg(fps, fpsynth, args)

    # ---------------- batch clustering search ----------------
    if "cluster" in legs:
        out["cluster"] = cluster_leg(lib, lib_np, fps, fpsynth)

    # ---------------- library file ingest ----------------
    if "ingest" in legs:
        out["ingest"] = ingest_leg(lib, lib_np, strides, fps, fpsynth)

    # ---------------- CPU baseline (oracle) ----------------
    if "cpu" in legs:
        out["cpu_baseline"] = cpu_baseline(lib_np, qs, args, fpsynth)

    if parity:
        out["parity"] = parity
    value = single["gcmp_s"] if single else None
    line = {
        "metric": "G fp-compares/s at 95.4M lib (1 & 1024 queries) + %HBM peak; p50/p99 latency",
        "value": value, "unit": "G fp-compares/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": single["ms_per_query"] if single else None,
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic (fpsynth MACCS-166-shaped, seed 1)",
        "config": {"workload": "single query top-30 over 95,417,114 fingerprints",
                   "n": n, "k": 30, "queries_per_step": 1,
                   "strides": strides},
    }
    line.update(out)
    if single:
        line["single"] = single
    print(json.dumps(line), flush=True)
    lib.close()


def wide_leg(fps, fpsynth, args):
    """Wider fingerprints (Section 5, concluding remark 3): 2,048 keys (32 words,
    256 bytes) per record, every bit a key.  One query, top-30, end to end
    through fps_wide_search; the scan kernel's duration from HIP events gives
    its HBM roofline (256 bytes per record compared).  Then 256 queries in one
    call on the fp4 matrix cores (2 x 2,048 operations per pair)."""
    import torch
    W, n = 32, args.wide_n
    t = time.perf_counter()
    lib_np = fpsynth.make_wide_library(n, W, 1, keep_meta=False)
    gen_s = time.perf_counter() - t
    lib = fps.WideLibrary(lib_np.words)
    qs, _, _ = fpsynth.make_wide_queries(lib_np, 23, 2001, flips=(0, 8), fresh=np.zeros(23))
    for i in range(3):
        lib.search(qs[i], 30)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(3, 23):
        lib.search(qs[i], 30)
    ms = (time.perf_counter() - t) * 1000 / 20
    lib.set_timing(True)
    s0 = lib.last_stats()
    for i in range(3, 23):
        lib.search(qs[i], 30)
    s1 = lib.last_stats()
    scan_ms = (s1["scan_ms_sum"] - s0["scan_ms_sum"]) / 20
    rec_bytes = 8 * W
    gbs = rec_bytes * n / (scan_ms * 1e-3) / 1e9
    r = {"records": n, "keys": 64 * W, "bytes_per_record": rec_bytes, "k": 30,
         "library_gb": rec_bytes * n / 1e9, "generate_s": gen_s,
         "ms_per_query": ms, "gcmp_s": n / (ms * 1e-3) / 1e9, "scan_ms_per_query": scan_ms,
         "scan_launches_per_query": s1["scan_launches"],
         "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": gbs / HBM_PEAK_GBS, "kernel": "k_wscan1<32>"}}
    # a batch on the matrix cores
    bq, _, _ = fpsynth.make_wide_queries(lib_np, 256, 2003)
    lib.set_path(fps.PATH_MFMA_F4)
    lib.search_batch(bq, 30)
    tb = []
    for _ in range(3):
        t = time.perf_counter()
        lib.search_batch(bq, 30)
        tb.append(time.perf_counter() - t)
    st = lib.last_stats()
    bms = float(np.median(tb)) * 1000
    tops = 2 * 64 * W * 256.0 * n / (st["scan_ms"] * 1e-3) / 1e12
    r["batch256"] = {"queries": 256, "path": st["path"], "ms": bms, "qps": 256 / (bms * 1e-3),
                     "scan_ms": st["scan_ms"], "speedup_vs_single_qps": ms * 256 / bms,
                     "roofline": {"bound": "mfma", "achieved": tops, "peak": FP4_PEAK_TFLOPS,
                                  "unit": "TFLOP/s", "frac": tops / FP4_PEAK_TFLOPS,
                                  "dtype": "fp4"}}
    lib.close()
    del lib_np
    torch.cuda.empty_cache()
    log("wide:", json.dumps(r))
    return r


def cluster_leg(lib, lib_np, fps, fpsynth):
    """Batch clustering search (Section 4.4, Fig. 2): the 1024-query batch
    clustered for every count 2..8 (k-medians, silhouette), then the top-30 of
    every chosen center over the whole library."""
    import torch
    q = fpsynth.batch_queries(lib_np, 1024, 1003).words
    fps.cluster(q, 2, 8)  # warm-up
    torch.cuda.synchronize()
    tc = []
    for _ in range(5):
        t = time.perf_counter()
        res = fps.cluster(q, 2, 8)
        tc.append(time.perf_counter() - t)
    lib.cluster_search(q, 30, 2, 8)
    ts = []
    for _ in range(5):
        t = time.perf_counter()
        full = lib.cluster_search(q, 30, 2, 8)
        ts.append(time.perf_counter() - t)
    r = {"queries": 1024, "k": 30, "counts_tried": [2, 8], "chosen_k": res["K"],
         "rounds": res["rounds"], "scores": {str(k): v for k, v in res["scores"].items()},
         "cluster_ms": float(np.median(tc)) * 1000,
         "cluster_search_ms": float(np.median(ts)) * 1000,
         "same_clustering_in_search": bool(np.array_equal(full["labels"], res["labels"]))}
    log("cluster:", json.dumps(r))
    return r


def ingest_leg(lib, lib_np, strides, fps, fpsynth):
    """The library file of Fig. 3 step 1 (one '<CID> <167 key characters>' line
    per molecule) parsed on the GPU from HBM into the packed library and its id
    column.  The text is copied to the GPU first (timed separately: the PCIe
    leg); the timed call counts the lines, then parses and validates every
    line, the id column staying in HBM (hits are mapped to ids on the device).
    One more load also downloads the ids to the host (timed on its own).  The
    result is checked against the library uploaded from the words and against
    the generated ids."""
    import torch
    n = lib_np.n
    t = time.perf_counter()
    ids = fpsynth.make_cids(n, 1)
    text = fpsynth.library_text(lib_np.words, ids)
    gen_s = time.perf_counter() - t
    nbytes = int(text.nbytes)
    torch.cuda.synchronize()
    t = time.perf_counter()
    dtext = torch.from_numpy(text).to("cuda")
    torch.cuda.synchronize()
    h2d_s = time.perf_counter() - t
    del text
    runs = []
    tl = None
    for r in range(3):
        if tl is not None:
            tl.close()
            tl = None
        torch.cuda.synchronize()
        t = time.perf_counter()
        tl = fps.Library(text=dtext, strides=strides, host_ids=False)
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t)
    dev_ids = tl.ids_device.cpu().numpy().astype(np.uint64)
    exact = bool(torch.equal(tl._buf, lib._buf)) and bool(np.array_equal(dev_ids, ids))
    del dev_ids
    tl.close()
    torch.cuda.synchronize()
    t = time.perf_counter()
    tl = fps.Library(text=dtext, strides=strides, host_ids=True)
    torch.cuda.synchronize()
    with_download_s = time.perf_counter() - t
    exact = exact and bool(np.array_equal(tl.ids, ids))
    sec = float(np.median(runs))
    r = {"records": n, "text_bytes": nbytes, "bytes_per_line": nbytes / n,
         "s_per_load": sec, "s_per_load_min": float(min(runs)),
         "text_gbs": nbytes / sec / 1e9, "lines_per_s": n / sec,
         "h2d_s": h2d_s, "h2d_gbs": nbytes / h2d_s / 1e9,
         "pcie_inclusive_gbs": nbytes / (h2d_s + sec) / 1e9,
         "generate_s": gen_s, "exact_vs_words_and_ids": exact,
         "s_per_load_with_id_download": with_download_s,
         "what": "fps_text_count + fps_text_library_load (count, prefix, parse and validate "
                 "every line; ids kept in HBM) on text already in HBM; with_id_download: "
                 "the same plus the id column copied to pageable host memory; h2d = pageable "
                 "copy"}
    tl.close()
    del dtext
    torch.cuda.empty_cache()
    log("ingest:", json.dumps(r))
    return r


def small_leg(fps, fpsynth, args):
    """100,000 records, top-30: the library fits the GPU's caches, so the figure
    is latency in microseconds, end to end through fps_search."""
    lib_np = fpsynth.make_library(100_000, 1)
    lib = fps.Library(lib_np.words)
    nq = 200
    qs = fpsynth.make_queries(lib_np, nq + 10, 1001, flips=(2, 2)).words
    for i in range(10):
        lib.search(qs[i], 30)
    per = []
    for i in range(10, 10 + nq):
        t = time.perf_counter()
        lib.search(qs[i], 30)
        per.append(time.perf_counter() - t)
    per = np.array(per) * 1e6
    r = {"records": 100_000, "k": 30, "queries": nq, "us_median": float(np.median(per)),
         "us_p99": float(np.percentile(per, 99)), "us_min": float(per.min()),
         "gcmp_s": 100_000 / (np.median(per) * 1e-6) / 1e9}
    lib.close()
    log("small:", json.dumps(r))
    return r


def serve(lib, lib_np, args, fps, fpsynth):
    import torch
    res = {}
    rates = [float(x) for x in args.serve_rates.split(",") if x]
    cfg = dict(pool_bytes=6 << 30, max_batch_queries=1024, n_streams=3, deadline_cap=True,
               reserve_streams=1)
    # the server tunes every batch shape of 1..1024 queries with each k at
    # creation, so no request waits for the autotuner
    t = time.perf_counter()
    srv = fps.Server(lib, tune_k=[30, 100, 1000], **cfg)
    log(f"server created, batch shapes tuned in {time.perf_counter() - t:.1f}s")
    for rate in rates:
        arr, sizes, ks = fpsynth.poisson_requests(rate, args.serve_seconds, 1005)
        nreq = len(arr)
        allq = fpsynth.batch_queries(lib_np, int(sizes.sum()), 1006).words
        offs = np.concatenate([[0], np.cumsum(sizes)])
        srv.stats(reset=True)
        t0 = fps.clock_ns() + 5_000_000
        sched = t0 + np.round(arr * 1e9).astype(np.int64)
        tickets = [None] * nreq
        rstats = [None] * nreq
        ready = threading.Semaphore(0)

        def waiter():
            for i in range(nreq):
                ready.acquire()
                _, _, rs = srv.wait(tickets[i])
                rstats[i] = rs

        th = threading.Thread(target=waiter)
        th.start()
        # Requests go in at their scheduled times and carry those times as
        # their arrivals: when admission blocks (the pool is full), later
        # requests are submitted late but their latency still starts at their
        # arrival.
        for i in range(nreq):
            now = fps.clock_ns()
            if sched[i] > now:
                time.sleep((sched[i] - now) * 1e-9)
            tickets[i] = srv.submit(allq[offs[i]:offs[i + 1]], int(ks[i]), fps.MASK_ALL,
                                    deadline_us=10_000, arrival_ns=int(sched[i]))
            ready.release()
        th.join()
        st = srv.stats()
        torch.cuda.synchronize()
        arrival = np.array([r["arrival_ns"] for r in rstats], dtype=np.int64)
        admit = np.array([r["submit_ns"] for r in rstats], dtype=np.int64)
        done = np.array([r["done_ns"] for r in rstats], dtype=np.int64)
        meas = arr >= args.serve_warmup
        win = (args.serve_seconds - args.serve_warmup)
        lat = (done - arrival)[meas] / 1e6
        wait_adm = (admit - arrival)[meas] / 1e6
        t_first = int(t0 + args.serve_warmup * 1e9)
        span_done = (done[meas].max() - t_first) / 1e9
        span_adm = (admit[meas].max() - t_first) / 1e9
        nmeas = int(meas.sum())
        qmeas = int(sizes[meas].sum())
        r = {"offered_req_s": rate, "requests": nmeas, "queries": qmeas,
             "offered_queries_s": qmeas / win,
             "admitted_req_s": nmeas / span_adm, "completed_req_s": nmeas / span_done,
             "completed_queries_s": qmeas / span_done,
             "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
             "max_ms": float(lat.max()),
             "admission_wait_p50_ms": float(np.percentile(wait_adm, 50)),
             "admission_wait_p99_ms": float(np.percentile(wait_adm, 99)),
             "deadline_miss_rate": float((lat > 10.0).mean()),
             "latency_from": "scheduled arrival", "seconds_of_arrivals": args.serve_seconds,
             "warmup_s": args.serve_warmup,
             "mean_batch_queries": st["mean_batch_queries"], "batches": int(st["batches"]),
             "untuned_batches": int(st["untuned_batches"]),
             "n_streams": cfg["n_streams"], "reserve_streams": cfg["reserve_streams"],
             "max_batch_queries": cfg["max_batch_queries"], "deadline_cap": True,
             "service_model_us": [round(st["cost_fixed_us"], 1),
                                  round(st["cost_per_weight_us"], 3)]}
        res[str(int(rate))] = r
        log("serve:", json.dumps(r))
    srv.close()
    return res


def cpu_baseline(lib_np, qs, args, fpsynth):
    import oracle
    nth = max(1, min(16, os.cpu_count() or 1))
    n = lib_np.n
    strides = [0, min(40_000_000, n), min(75_000_000, n), n]

    def timed(queries, ks, masks, budget):
        t = time.perf_counter()
        recs = 0
        done = 0
        for q, k, m in zip(queries, ks, masks):
            rr = oracle.mask_ranges(strides, m)
            oracle.search(lib_np.words, q, int(k), ranges=rr, nthreads=nth)
            recs += sum(e - b for b, e in rr)
            done += 1
            if time.perf_counter() - t > budget:
                break
        return recs, done, time.perf_counter() - t

    # single queries of the headline workload
    rs, ds, es = timed(qs, [30] * len(qs), [None] * len(qs), args.cpu_seconds)
    # a stratified subset of the 1024-query batch: library-derived and fresh
    # queries alternate
    bq = fpsynth.batch_queries(lib_np, 1024, 1003).words
    rb, db, eb = timed(bq[:8], [30] * 8, [None] * 8, args.cpu_seconds)
    # the uneven batch: one query of every (k, mask) combination
    uq = fpsynth.batch_queries(lib_np, 4096, 1004).words
    uk, um = fpsynth.uneven_params(4096, 1004)
    picks = []
    for kk in fpsynth.K_CHOICES:
        for mm in fpsynth.MASK_CHOICES:
            idx = np.nonzero((uk == kk) & (um == mm))[0]
            if len(idx):
                picks.append(int(idx[0]))
    ru, du, eu = timed(uq[picks], uk[picks], um[picks], 2 * args.cpu_seconds)
    # the plain serial form on one core, over the first eighth of the library
    n1 = max(1, n // 8)
    t1 = time.perf_counter()
    oracle.search(lib_np.words[:n1], qs[0], 30, nthreads=1)
    el1 = time.perf_counter() - t1
    # batch clustering of the 1024-query batch (counts 2..8), the oracle's form
    import oracle.cluster as ocl
    tcl = time.perf_counter()
    ocl.cluster(bq, 2, 8)
    ecl = time.perf_counter() - tcl
    r = {"value": rs / es / 1e9, "unit": "G fp-compares/s", "cores": nth,
         "kind": "oracle",
         "sample": f"{ds} full-library single queries (top-30 over {n} records), "
                   f"threaded chunk-and-merge form, {es:.1f}s wall",
         "batch1024": {"value": rb / eb / 1e9,
                       "sample": f"queries 0..{db - 1} of the 1024-query set (library-derived "
                                 f"and fresh alternate), top-30, {eb:.1f}s",
                       "queries_s": db / eb},
         "uneven4096": {"value": ru / eu / 1e9,
                        "sample": f"{du} queries, the first of each (k, mask) combination of "
                                  f"the 4096-query set, {eu:.1f}s",
                        "queries_s": du / eu},
         "one_core": {"value": n1 / el1 / 1e9, "sample": f"one query over {n1} records, "
                                                         f"serial form, {el1:.1f}s"},
         "cluster1024": {"seconds": ecl, "sample": "clustering of the whole 1024-query batch "
                                                   "for counts 2..8 (oracle/cluster.py)"},
         "cpu_model": cpu_model(), "cpu_ident": cpu_ident(), "host_cpus": os.cpu_count()}
    log("cpu:", json.dumps(r))
    return r


if __name__ == "__main__":
    main()
