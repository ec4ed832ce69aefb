"""CPU ORACLE -- test infrastructure, not part of the product.

Batch clustering search (Section 4.4: a batch of fingerprints is clustered and
the top 30 molecules are found per cluster; Fig. 2: the number of clusters
("categories") is chosen by the silhouette ("contour") coefficient).  The paper
names neither the clustering algorithm nor what is searched for a category;
the reading taken, step by step, in the paper's Manhattan distance (Section
4.3):

  1. pairwise distances D[i][j] of the Q batch fingerprints;
  2. for every cluster count K in [k_min, k_max] (k_max < Q):
       a. initial centers by farthest-first traversal: center 0 is fingerprint
          0; center c is the fingerprint farthest from its nearest chosen
          center (ties: lowest index);
       b. k-medians (Lloyd iterations under the Manhattan distance): every
          fingerprint joins its nearest center (ties: lowest center index);
          every center becomes the key-wise majority of its members (key set
          iff more than half of the members have it; an empty cluster keeps
          its center) -- the key-wise median, which minimises the summed
          Manhattan distance to the members; repeat until no label changes,
          at most max_iter rounds;
       c. silhouette (Rousseeuw, J. Comput. Appl. Math. 20, 1987) of every
          fingerprint: a = mean distance to the other members of its cluster,
          b = smallest mean distance to the members of another cluster,
          s = (b - a) / max(a, b); s = 0 for a member of a singleton cluster
          or when max(a, b) = 0; the score of K is the mean of s, summed in
          index order in float64;
  3. K* = the K of the largest score (ties: the smaller K);
  4. for each of the K* clusters, the top-k library records nearest to its
     center (Fig. 3 with the center as the target), ascending (distance,
     index).

Every distance here is the oracle's key-by-key Section 4.3 sum (oracle.c).
Float64 enters only in step 2c; each s is computed by the same four IEEE
operations on exact integer sums, so an implementation doing the same
operations gets the same bits.  Pinned by tests/test_oracle_cluster.py.
"""
from __future__ import annotations

import numpy as np

import oracle

KEYS = 166


def _rows(words) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(words, dtype=np.uint64).reshape(-1, 3))


def pair_distances(queries) -> np.ndarray:
    """Step 1: D[i][j] = Section 4.3 distance of fingerprints i and j."""
    q = _rows(queries)
    n = len(q)
    D = np.zeros((n, n), dtype=np.int64)
    for i in range(n):
        D[i] = oracle.distances(q, q[i])
    return D


def key_bits(words) -> np.ndarray:
    """(n, 167) 0/1 matrix: column j is key j (column 0 is always 0)."""
    w = _rows(words)
    bits = np.unpackbits(w.view(np.uint8), axis=1, bitorder="little")
    return bits[:, :KEYS + 1].astype(np.int64)


def pack_bits(bits) -> np.ndarray:
    """Inverse of key_bits for one row."""
    v = 0
    for j in range(1, KEYS + 1):
        if bits[j]:
            v |= 1 << j
    return np.array([(v >> (64 * w)) & ((1 << 64) - 1) for w in range(3)], dtype=np.uint64)


def farthest_first(D: np.ndarray, K: int) -> list:
    """Step 2a: indices of the initial centers."""
    centers = [0]
    near = D[0].copy()
    while len(centers) < K:
        far = int(np.argmax(near))  # argmax returns the lowest index of the maximum
        centers.append(far)
        near = np.minimum(near, D[far])
    return centers


def k_medians(queries, K: int, max_iter: int = 100, D=None):
    """Step 2a-b: (labels (Q,), centers (K, 3) words, rounds run)."""
    q = _rows(queries)
    if D is None:
        D = pair_distances(q)
    centers = q[farthest_first(D, K)].copy()
    bits = key_bits(q)
    labels = None
    rounds = 0
    for rounds in range(1, max_iter + 1):
        # assignment: nearest center, ties to the lowest center index
        dc = np.stack([oracle.distances(q, centers[c]) for c in range(K)], axis=1)
        new = np.argmin(dc, axis=1)
        changed = labels is None or not np.array_equal(new, labels)
        labels = new
        # update: key-wise strict majority of the members
        for c in range(K):
            members = bits[labels == c]
            if len(members) == 0:
                continue
            counts = members.sum(axis=0)
            centers[c] = pack_bits(2 * counts > len(members))
        if not changed:
            break
    return labels.astype(np.int64), centers, rounds


def silhouette_values(D: np.ndarray, labels: np.ndarray, K: int) -> np.ndarray:
    """Step 2c: s of every fingerprint (float64)."""
    n = len(labels)
    size = np.bincount(labels, minlength=K)
    s = np.zeros(n, dtype=np.float64)
    for i in range(n):
        own = int(labels[i])
        if size[own] <= 1:
            continue
        # integer distance sums per cluster (exact: float64 holds them exactly)
        sums = [int(x) for x in np.bincount(labels, weights=D[i], minlength=K)]
        a = float(sums[own]) / float(size[own] - 1)
        b = None
        for c in range(K):
            if c != own and size[c] > 0:
                m = float(sums[c]) / float(size[c])
                b = m if b is None or m < b else b
        if b is None:
            continue
        top = max(a, b)
        if top > 0.0:
            s[i] = (b - a) / top
    return s


def silhouette_score(D, labels, K) -> float:
    s = silhouette_values(D, labels, K)
    tot = 0.0
    for x in s:  # index order, one addition at a time
        tot += float(x)
    return tot / float(len(s))


def cluster(queries, k_min: int = 2, k_max: int = 8, max_iter: int = 100):
    """Steps 1-3: dict with K (the chosen count), labels, centers, rounds and
    score[K] for every K tried."""
    q = _rows(queries)
    D = pair_distances(q)
    k_max = min(k_max, len(q) - 1)
    best = None
    scores = {}
    for K in range(k_min, k_max + 1):
        labels, centers, rounds = k_medians(q, K, max_iter, D)
        sc = silhouette_score(D, labels, K)
        scores[K] = sc
        if best is None or sc > best[0]:
            best = (sc, K, labels, centers, rounds)
    _, K, labels, centers, rounds = best
    return {"K": K, "labels": labels, "centers": centers, "rounds": rounds, "scores": scores}


def cluster_search(lib_words, queries, k: int = 30, k_min: int = 2, k_max: int = 8,
                   ranges=None, max_iter: int = 100, nthreads: int = 1):
    """Step 4: the clustering of `cluster` plus the top-k of every center."""
    res = cluster(queries, k_min, k_max, max_iter)
    res["hits"] = [oracle.search(lib_words, c, k, ranges=ranges, nthreads=nthreads)
                   for c in res["centers"]]
    return res
