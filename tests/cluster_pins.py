"""Pins of the oracle's batch clustering search (oracle/cluster.py) against
facts that do not use its code: brute-force definitions in plain Python
integers, the silhouette of scikit-learn (a library routine), the median
property of the key-wise majority, and planted clusters that must be found.
Each pin takes the module under test (the real one, or a copy with a planted
mistake)."""
from __future__ import annotations

import random

import numpy as np

import fpsynth
import oracle

KEYS = range(1, 167)


def as_int(rec) -> int:
    r = [int(x) for x in np.asarray(rec, dtype=np.uint64).reshape(3)]
    return r[0] | (r[1] << 64) | (r[2] << 128)


def from_int(v: int) -> np.ndarray:
    return np.array([(v >> (64 * w)) & ((1 << 64) - 1) for w in range(3)], dtype=np.uint64)


def d(a, b) -> int:
    return (as_int(a) ^ as_int(b)).bit_count()


def planted(groups, size, flips, seed):
    """`groups` random centers at least 40 keys apart, `size` members each with
    up to `flips` distinct flipped keys; returns (queries, group of each)."""
    rnd = random.Random(seed)
    cents = []
    while len(cents) < groups:
        c = sum(1 << j for j in rnd.sample(list(KEYS), 45))
        if all((c ^ o).bit_count() >= 40 for o in cents):
            cents.append(c)
    qs, grp = [], []
    for g, c in enumerate(cents):
        for _ in range(size):
            v = c
            for j in rnd.sample(list(KEYS), rnd.randint(0, flips)):
                v ^= 1 << j
            qs.append(from_int(v))
            grp.append(g)
    order = list(range(len(qs)))
    rnd.shuffle(order)
    return np.stack([qs[i] for i in order]), np.array([grp[i] for i in order])


def pin_pair_distances(cl):
    q = fpsynth.batch_queries(fpsynth.make_library(2000, 3), 60, 8).words
    D = cl.pair_distances(q)
    for i in range(60):
        for j in range(60):
            assert D[i][j] == d(q[i], q[j])


def pin_farthest_first(cl):
    rnd = random.Random(5)
    for t in range(20):
        q = fpsynth.batch_queries(fpsynth.make_library(500, t + 1), 25, t).words
        D = cl.pair_distances(q)
        K = rnd.randint(2, 8)
        want = [0]
        while len(want) < K:
            best, bi = -1, -1
            for i in range(len(q)):
                near = min(d(q[i], q[c]) for c in want)
                if near > best:
                    best, bi = near, i
            want.append(bi)
        assert cl.farthest_first(D, K) == want


def pin_kmedians_fixed_point(cl):
    for seed in (1, 2, 3):
        q = fpsynth.batch_queries(fpsynth.make_library(5000, seed), 200, seed + 40).words
        for K in (2, 3, 5, 8):
            labels, centers, rounds = cl.k_medians(q, K)
            assert rounds < 100
            ints = [as_int(x) for x in q]
            cint = [as_int(c) for c in centers]
            for i, v in enumerate(ints):
                ds = [(v ^ c).bit_count() for c in cint]
                assert labels[i] == ds.index(min(ds)), (seed, K, i)
            for c in range(K):
                members = [ints[i] for i in range(len(ints)) if labels[i] == c]
                if not members:
                    continue
                maj = 0
                for j in KEYS:
                    if 2 * sum((m >> j) & 1 for m in members) > len(members):
                        maj |= 1 << j
                assert cint[c] == maj, (seed, K, c)
                # the majority is a median: no member and no single-key change
                # of it has a smaller summed distance
                cost = sum((m ^ maj).bit_count() for m in members)
                for y in members[:20]:
                    assert cost <= sum((m ^ y).bit_count() for m in members)
                for j in list(KEYS)[::7]:
                    y = maj ^ (1 << j)
                    assert cost <= sum((m ^ y).bit_count() for m in members)


def pin_silhouette_library(cl):
    from sklearn.metrics import silhouette_samples
    for seed in (4, 5):
        q = fpsynth.batch_queries(fpsynth.make_library(5000, seed), 150, seed).words
        bits = np.unpackbits(np.ascontiguousarray(q).view(np.uint8), axis=1,
                             bitorder="little")[:, 1:167].astype(np.int64)
        D = cl.pair_distances(q)
        for K in (2, 4, 7):
            labels, _, _ = cl.k_medians(q, K)
            if len(set(labels.tolist())) < 2:
                continue
            want = silhouette_samples(bits, labels, metric="manhattan")
            got = cl.silhouette_values(D, labels, K)
            assert np.allclose(got, want, rtol=0, atol=1e-12), (seed, K)
    # singleton clusters and identical fingerprints score 0
    q = np.stack([from_int(0), from_int(0), from_int(2), from_int(2 | 4 | 8)])
    D = cl.pair_distances(q)
    s = cl.silhouette_values(D, np.array([0, 0, 1, 2]), 3)
    assert s[2] == 0.0 and s[3] == 0.0 and s[0] == 1.0 and s[1] == 1.0


def pin_planted_clusters(cl):
    for groups, size, seed in ((2, 30, 1), (3, 20, 2), (5, 12, 3), (7, 9, 4)):
        q, grp = planted(groups, size, 3, seed)
        res = cl.cluster(q, 2, 8)
        assert res["K"] == groups, (groups, res["scores"])
        # the partition is the planted one (labels up to renaming)
        pairs = set(zip(res["labels"].tolist(), grp.tolist()))
        assert len(pairs) == groups
        assert res["scores"][groups] == max(res["scores"].values())


def pin_equal_scores_take_smallest_k(cl):
    # identical fingerprints: every K scores 0, and the smallest K is taken
    q = np.stack([from_int((1 << 5) | (1 << 99))] * 6)
    res = cl.cluster(q, 2, 5)
    assert all(v == 0.0 for v in res["scores"].values())
    assert res["K"] == 2 and res["labels"].tolist() == [0] * 6


def pin_cluster_search(cl):
    lib = fpsynth.make_library(20_000, 9)
    q, _ = planted(3, 10, 2, 11)
    res = cl.cluster_search(lib.words, q, 30, 2, 5)
    assert len(res["hits"]) == res["K"]
    for c, h in enumerate(res["hits"]):
        want = oracle.search(lib.words, res["centers"][c], 30)
        assert np.array_equal(h, want)
        assert np.all(np.diff(h["distance"].astype(np.int64)) >= 0)


ALL_CLUSTER_PINS = [pin_pair_distances, pin_farthest_first, pin_kmedians_fixed_point,
                    pin_silhouette_library, pin_planted_clusters,
                    pin_equal_scores_take_smallest_k, pin_cluster_search]
