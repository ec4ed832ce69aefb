#!/usr/bin/env python3
"""Benchmark of the exact MACCS-166 top-k engine on one MI355X.

Headline (value): one query, top-30, against 95,417,114 synthetic MACCS-shaped
fingerprints resident in HBM -- the library size and k of the paper (Section
2.2, Fig. 2) -- in G fingerprint comparisons per second, end to end through
fps_search (query upload, bound, scan, select, result download).  Every step
uses a different query (a library record with 0-5 flipped keys).

Also measured in the same run (secondary objects of the JSON line):
  batch   : 1024 queries (half library records with 1-8 flips, half fresh), k = 30
  uneven  : 4096 queries, k uniform over {1,10,30,100,1000}, masks over
            {A, A+B, A+B+C} of strides 40M / 35M / 20.4M
  serving : Poisson request arrivals, 1-64 queries per request, k in
            {30,100,1000}, 10 ms deadline; p50 / p99 latency and throughput over
            the arrivals after a 1 s warm-up (6 s per rate)
  cpu_baseline : the CPU oracle on the host's cores, on a bounded sample.

Inputs are synthetic (fpsynth): the PubChem library of the paper is not
available.  One JSON line is printed on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# HBM traffic of the single-query scan kernel, from two rocprofv3 counter runs
# (FETCH_SIZE, WRITE_SIZE) scaled by a calibration copy; valid only while the
# kernel sources hash to what the summary records.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_scan_single.single_top30_95M.hbm_traffic.txt")
TRAFFIC_SOURCES = ["paper_1906_06170_amd/csrc/kernels.hip", "paper_1906_06170_amd/csrc/cand.h",
                   "paper_1906_06170_amd/csrc/fps_internal.h"]


def measured_traffic():
    import hashlib
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=95_417_114)
    ap.add_argument("--only", default="all",
                    help="comma list of: single,shard,batch,uneven,serve,cpu")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--serve-seconds", type=float, default=6.0)
    ap.add_argument("--serve-warmup", type=float, default=1.0,
                    help="seconds of arrivals per rate excluded from the statistics")
    ap.add_argument("--serve-rates", default="200,1000,5000")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
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
        "single", "shard", "batch", "uneven", "serve", "cpu"}

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

    t0 = time.time()
    n = args.n
    strides = [0, min(40_000_000, n), min(75_000_000, n), n]
    lib_np = fpsynth.make_library(n, 1, keep_meta=False)
    log(f"library: {n} records generated in {time.time() - t0:.1f}s")
    t1 = time.time()
    lib = fps.Library(lib_np.words, strides=strides)
    log(f"uploaded in {time.time() - t1:.1f}s")
    out = {}

    # ---------------- single query ----------------
    K, W = args.steps, args.warmup
    qs = fpsynth.make_queries(lib_np, K + W, 1001, flips=(0, 5)).words
    single = None
    if "single" in legs:
        for i in range(W):
            lib.search(qs[i], 30)
        torch.cuda.synchronize()
        # the timed steps run untimed on the device (no HIP events) ...
        per_q = []
        t = time.perf_counter()
        for i in range(W, W + K):
            tq = time.perf_counter()
            lib.search(qs[i], 30)  # synchronous: returns with the hits on the host
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
        }
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": measured_traffic(),
                           "kernel": "k_scan_single",
                           "bytes_per_launch": ALGO_BYTES_PER_RECORD * n / max(1, launches / K),
                           "launch_avg_ms": scan_ms / max(1, launches)}
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
        bq = fpsynth.batch_queries(lib_np, 1024, 1003).words
        lib.set_path(path)
        lib.set_timing(True)  # events cost microseconds against a multi-ms batch
        for _ in range(2):  # first sight: autotuner; second: graph capture
            lib.search_batch(bq, 30)
        torch.cuda.synchronize()
        times, scans = [], []
        for _ in range(args.batch_steps):
            t = time.perf_counter()
            lib.search_batch(bq, 30)
            times.append(time.perf_counter() - t)
            scans.append(lib.last_stats())
        ms = float(np.median(times)) * 1000
        scan = float(np.median([s["scan_ms"] for s in scans]))
        pairs = 1024 * n
        b = {"queries": 1024, "k": 30, "path": scans[-1]["path"], "ms": ms,
             "qps": 1024 / (ms * 1e-3), "gcmp_s": pairs / (ms * 1e-3) / 1e9,
             "scan_kernel_ms": scan, "candidates": scans[-1]["candidates"],
             "fallbacks": scans[-1]["fallbacks"], "variant": scans[-1]["variant"],
             "graph_replay": scans[-1]["graph"]}
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
        out["batch"] = b
        lib.set_path(fps.PATH_AUTO)
        lib.set_timing(False)
        log("batch:", json.dumps(b))

    # ---------------- uneven 4096 ----------------
    if "uneven" in legs:
        uq = fpsynth.batch_queries(lib_np, 4096, 1004).words
        uk, um = fpsynth.uneven_params(4096, 1004)
        lib.set_path(path)
        lib.set_timing(True)
        for _ in range(2):
            lib.search_batch(uq, uk, um)
        times, scans = [], []
        for _ in range(max(2, args.batch_steps // 2)):
            t = time.perf_counter()
            lib.search_batch(uq, uk, um)
            times.append(time.perf_counter() - t)
            scans.append(lib.last_stats())
        ms = float(np.median(times)) * 1000
        neff = {1: strides[1], 3: strides[2], 7: n}
        pairs = int(sum(neff[int(m)] for m in um))
        u = {"queries": 4096, "path": scans[-1]["path"], "ms": ms,
             "qps": 4096 / (ms * 1e-3), "gcmp_s": pairs / (ms * 1e-3) / 1e9,
             "scan_kernel_ms": float(np.median([s["scan_ms"] for s in scans])),
             "fallbacks": scans[-1]["fallbacks"]}
        out["uneven"] = u
        lib.set_path(fps.PATH_AUTO)
        lib.set_timing(False)
        log("uneven:", json.dumps(u))

    # ---------------- serving ----------------
    if "serve" in legs:
        out["serving"] = serve(lib, lib_np, args, fps, fpsynth)

    # ---------------- CPU baseline (oracle) ----------------
    if "cpu" in legs:
        out["cpu_baseline"] = cpu_baseline(lib_np, qs, args)

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


def serve(lib, lib_np, args, fps, fpsynth):
    import torch
    res = {}
    # warm-up outside the timed window: the autotuner times the kernels once per
    # batch shape (queries and largest k, each rounded up to a power of two)
    t = time.perf_counter()
    wq = fpsynth.batch_queries(lib_np, 1024, 999).words
    for k in (30, 100, 1000):
        nq = 1
        while nq <= 1024:
            lib.search_batch(wq[:nq], k)
            nq *= 2
    log(f"serving warm-up (autotuner) {time.perf_counter() - t:.1f}s")
    rates = [float(x) for x in args.serve_rates.split(",") if x]
    for rate in rates:
        arr, sizes, ks = fpsynth.poisson_requests(rate, args.serve_seconds, 1005)
        nreq = len(arr)
        allq = fpsynth.batch_queries(lib_np, int(sizes.sum()), 1006).words
        offs = np.concatenate([[0], np.cumsum(sizes)])
        srv = fps.Server(lib, pool_bytes=6 << 30, max_batch_queries=1024, n_streams=3,
                         deadline_cap=True, reserve_streams=1)
        tickets = [None] * nreq
        done = threading.Event()

        def waiter():
            for i in range(nreq):
                while tickets[i] is None:
                    time.sleep(50e-6)
                srv.wait(tickets[i], int(sizes[i]), int(ks[i]))
            done.set()

        th = threading.Thread(target=waiter)
        th.start()
        t0 = time.perf_counter()
        t_meas = None
        for i in range(nreq):
            delay = arr[i] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            if t_meas is None and arr[i] >= args.serve_warmup:
                srv.stats(reset=True)  # statistics cover arrivals after the warm-up
                t_meas = time.perf_counter()
            tickets[i] = srv.submit(allq[offs[i]:offs[i + 1]], int(ks[i]), fps.MASK_ALL,
                                    deadline_us=10_000)
        done.wait()
        el = time.perf_counter() - (t_meas if t_meas is not None else t0)
        th.join()
        st = srv.stats()
        srv.close()
        torch.cuda.synchronize()
        r = {"offered_req_s": rate, "requests": int(st["requests"]),
             "achieved_req_s": st["requests"] / el, "queries_s": st["queries"] / el,
             "p50_ms": st["p50_us"] / 1000, "p99_ms": st["p99_us"] / 1000,
             "max_ms": st["max_us"] / 1000, "deadline_miss_rate":
                 st["deadline_misses"] / max(1, st["requests"]),
             "mean_batch_queries": st["mean_batch_queries"], "batches": int(st["batches"]),
             "n_streams": 3, "reserve_streams": 1, "max_batch_queries": 1024,
             "deadline_cap": True,
             "service_model_us": [round(st["cost_fixed_us"], 1),
                                  round(st["cost_per_weight_us"], 3)]}
        res[str(int(rate))] = r
        log("serve:", json.dumps(r))
    return res


def cpu_baseline(lib_np, qs, args):
    import oracle
    nth = max(1, min(16, os.cpu_count() or 1))
    n = lib_np.n
    t = time.perf_counter()
    done = 0
    i = 0
    while True:
        oracle.search(lib_np.words, qs[i % len(qs)], 30, nthreads=nth)
        done += 1
        i += 1
        if time.perf_counter() - t > args.cpu_seconds or done >= 8:
            break
    el = time.perf_counter() - t
    # the plain serial form on one core, over the first eighth of the library
    n1 = max(1, n // 8)
    t1 = time.perf_counter()
    oracle.search(lib_np.words[:n1], qs[0], 30, nthreads=1)
    el1 = time.perf_counter() - t1
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    r = {"value": done * n / el / 1e9, "unit": "G fp-compares/s", "cores": nth,
         "kind": "oracle",
         "sample": f"{done} full-library single queries (top-30 over {n} records), "
                   f"threaded chunk-and-merge form, {el:.1f}s wall",
         "one_core": {"value": n1 / el1 / 1e9, "sample": f"one query over {n1} records, "
                                                         f"serial form, {el1:.1f}s"},
         "cpu_model": model, "host_cpus": os.cpu_count()}
    log("cpu:", json.dumps(r))
    return r


if __name__ == "__main__":
    main()
