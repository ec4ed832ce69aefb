"""The shared input generator: reproducibility and the model's structure."""
import numpy as np

import fpsynth
from pins import as_int, key_set


def test_same_seed_same_bytes():
    a = fpsynth.make_library(20_000, 7, nthreads=1)
    b = fpsynth.make_library(20_000, 7, nthreads=8)
    assert a.words.tobytes() == b.words.tobytes()
    assert np.array_equal(a.dup_src, b.dup_src)
    c = fpsynth.make_library(20_000, 8)
    assert a.words.tobytes() != c.words.tobytes()


def test_unused_bits_zero_and_density():
    lib = fpsynth.make_library(50_000, 3)
    v = [as_int(r) for r in lib.words[:5000]]
    assert all((x & 1) == 0 and (x >> 167) == 0 for x in v)
    w = lib.words
    assert not np.any(w[:, 0] & np.uint64(1))
    assert not np.any(w[:, 2] >> np.uint64(39))
    frac = np.mean([x.bit_count() for x in v]) / 166
    assert 0.15 < frac < 0.32


def test_near_duplicate_fraction_and_sources():
    lib = fpsynth.make_library(100_000, 1)
    d = lib.dup_src >= 0
    assert 0.045 < d.mean() < 0.055
    idx = np.nonzero(d)[0]
    assert np.all(lib.dup_src[idx] < idx)
    assert set(np.unique(lib.dup_flips[idx]).tolist()) == {0, 1, 2, 3}
    for i in idx[:500]:
        diff = key_set(lib.words[i]) ^ key_set(lib.words[lib.dup_src[i]])
        assert len(diff) == lib.dup_flips[i]


def test_query_kinds():
    lib = fpsynth.make_library(10_000, 2)
    qs = fpsynth.batch_queries(lib, 64, 1003)
    assert np.all(qs.src[1::2] == -1) and np.all(qs.src[0::2] >= 0)
    f = qs.flips[0::2]
    assert f.min() >= 1 and f.max() <= 8
    for q in range(0, 64, 2):
        assert len(key_set(qs.words[q]) ^ key_set(lib.words[qs.src[q]])) == qs.flips[q]
    one = fpsynth.make_queries(lib, 5, 1, flips=(2, 2))
    assert np.all(one.flips == 2)


def test_uneven_params_cover_choices():
    k, m = fpsynth.uneven_params(4096, 1004)
    assert set(k.tolist()) == set(fpsynth.K_CHOICES)
    assert set(m.tolist()) == set(fpsynth.MASK_CHOICES)
    assert fpsynth.PAPER_STRIDES == [0, 40_000_000, 75_000_000, 95_417_114]


def test_poisson_trace():
    t, sizes, ks = fpsynth.poisson_requests(1000.0, 2.0, 1005)
    assert abs(len(t) - 2000) < 200
    assert sizes.min() >= 1 and sizes.max() <= 64
    assert set(ks.tolist()) <= {30, 100, 1000}
    assert np.all(np.diff(t) >= 0)
