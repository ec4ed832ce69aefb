"""Batch clustering search (Section 4.4, Fig. 2) on the GPU against the oracle
(oracle/cluster.py): chosen cluster count, labels, centers, k-medians rounds
and every silhouette score must be equal -- the integer parts exactly, the
float64 scores bit for bit (both sides compute every score from the same
exact integer sums with the same IEEE operations in the same order) -- and
the top-k of every center equal to the oracle's search."""
import numpy as np
import pytest

import fpsynth
import oracle
import oracle.cluster as ocl
from cluster_pins import planted

fps = pytest.importorskip("paper_1906_06170_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def same_clustering(got, want, what=""):
    assert got["K"] == want["K"], (what, got["scores"], want["scores"])
    assert np.array_equal(got["labels"], want["labels"]), what
    assert np.array_equal(got["centers"], want["centers"]), what
    assert got["rounds"] == want["rounds"], what
    for K, v in want["scores"].items():
        assert got["scores"][K] == v, (what, K, got["scores"][K], v)


@pytest.mark.parametrize("groups,size,seed", [(2, 30, 1), (3, 20, 2), (5, 12, 3), (7, 9, 4)])
def test_planted_clusters_match_oracle(groups, size, seed):
    q, grp = planted(groups, size, 3, seed)
    say("case: planted", groups, size, seed)
    got = fps.cluster(q, 2, 8)
    want = ocl.cluster(q, 2, 8)
    same_clustering(got, want, f"planted {groups}")
    assert got["K"] == groups


@pytest.mark.parametrize("nq,kmin,kmax,seed", [(3, 2, 2, 1), (7, 2, 6, 2), (100, 2, 8, 3),
                                               (1024, 2, 8, 4), (1000, 3, 16, 5),
                                               (4096, 2, 8, 6)])
def test_random_batches_match_oracle(nq, kmin, kmax, seed):
    lib = fpsynth.make_library(20_000, seed)
    q = fpsynth.batch_queries(lib, nq, 700 + seed).words
    say("case: random batch", nq, kmin, kmax)
    got = fps.cluster(q, kmin, kmax)
    want = ocl.cluster(q, kmin, kmax)
    same_clustering(got, want, f"random {nq}")


def test_identical_and_duplicate_targets():
    one = fpsynth.make_library(3, 8).words
    q = np.concatenate([np.tile(one[0], (10, 1)), np.tile(one[1], (3, 1))])
    for qq in (np.tile(one[0], (6, 1)), q):
        got = fps.cluster(qq, 2, 5)
        want = ocl.cluster(qq, 2, 5)
        same_clustering(got, want, "duplicates")


def test_cluster_search_matches_oracle():
    n = 100_000
    lib_np = fpsynth.make_library(n, 2)
    strides = [0, 40_000, 75_000, n]
    lib = fps.Library(lib_np.words, strides=strides)
    q, _ = planted(4, 16, 3, 9)
    for k, mask in ((30, fps.MASK_ALL), (1000, 3), (1, 4)):
        say("case: cluster search k", k, "mask", mask)
        got = lib.cluster_search(q, k, 2, 8, mask)
        rr = None if mask == fps.MASK_ALL else oracle.mask_ranges(strides, mask)
        want = ocl.cluster_search(lib_np.words, q, k, 2, 8, ranges=rr)
        same_clustering(got, want, "search")
        assert len(got["hits"]) == want["K"]
        for c in range(want["K"]):
            assert np.array_equal(got["hits"][c], want["hits"][c]), (k, mask, c)


def test_cluster_argument_errors():
    q = fpsynth.batch_queries(fpsynth.make_library(100, 1), 10, 1).words
    for args in ((q[:2], 2, 2), (q, 1, 4), (q, 5, 4), (q, 2, 10), (q, 2, 17)):
        with pytest.raises(fps.FPSError) as e:
            fps.cluster(*args)
        assert e.value.status == fps.FPS_E_ARG
    bad = q.copy()
    bad[4, 0] |= np.uint64(1)
    with pytest.raises(fps.FPSError) as e:
        fps.cluster(bad, 2, 4)
    assert e.value.status == fps.FPS_E_FINGERPRINT
