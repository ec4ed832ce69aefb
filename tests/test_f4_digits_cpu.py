"""The fp4 digit arithmetic of the matrix-core scan (csrc/f4_digits.h), on the
host: every count and bias value the kernel can meet, and tiles of (query,
record) pairs laid out as the kernel's operand fragments, whose dot product
must be u = d - T - 1 with d the oracle's distance (the matrix form of the
Section 4.3 distance, d = |q| + |r| - 2 q.r, shifted by the bound)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import fpsynth
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1906_06170_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ALL_KEYS = (0xFFFFFFFFFFFFFFFE, 0xFFFFFFFFFFFFFFFF, (1 << 39) - 1)


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("no hipcc")
    exe = str(tmp_path_factory.mktemp("f4") / "f4_digits_check")
    subprocess.run([HIPCC, "--cuda-host-only", "-x", "hip", "-std=c++17", "-O1", "-Wall",
                    "-Werror", "-I", CSRC, os.path.join(ROOT, "tests", "f4_digits_check.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


def run(exe, rows, recs):
    lines = [f"{len(rows)} {len(recs)}"]
    lines += [f"{int(w[0])} {int(w[1])} {int(w[2])} {int(t)} {int(v)}" for w, t, v in rows]
    lines += [f"{int(w[0])} {int(w[1])} {int(w[2])} {int(v)}" for w, v in recs]
    out = subprocess.run([exe], input="\n".join(lines) + "\n", check=True, capture_output=True,
                         text=True).stdout
    res, u = {}, {}
    for line in out.splitlines():
        f = line.split()
        if f[0] == "u":
            u[(int(f[1]), int(f[2]))] = float(f[3])
        else:
            res[f[0]] = int(f[1])
    return res, u


def test_every_count_and_bias(checker):
    res, _ = run(checker, [], [])
    assert res == {"six_one_bad": 0, "pop_bad": 0, "bias_bad": 0}


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tile_products_are_shifted_distances(checker, seed):
    lib = fpsynth.make_library(5000, seed)
    rng = np.random.default_rng(seed)
    recs = [(lib.words[i], 1) for i in rng.choice(lib.n, 36, replace=False)]
    recs += [((0, 0, 0), 1), (ALL_KEYS, 1), (lib.words[0], 0), (ALL_KEYS, 0)]
    qw = list(fpsynth.batch_queries(lib, 30, 100 + seed).words)
    qw += [np.zeros(3, dtype=np.uint64), np.array(ALL_KEYS, dtype=np.uint64)]
    qw += [recs[0][0], recs[1][0]]  # distance 0 to a record of the tile
    t_cycle = [-1, 0, 1, 5, 20, 40, 80, 166]
    rows = []
    for i, w in enumerate(qw):
        t = t_cycle[i % len(t_cycle)] if i % 3 else int(rng.integers(0, 167))
        rows.append((w, t, 1))
    rows += [(qw[0], 166, 0), (np.zeros(3, dtype=np.uint64), -1, 0)]  # invalid rows
    _, u = run(checker, rows, recs)
    assert len(u) == len(rows) * len(recs)
    for qi, (w, t, qv) in enumerate(rows):
        for ri, (r, rv) in enumerate(recs):
            got = u[(qi, ri)]
            if qv and rv:
                d = oracle.distance(w, r)
                assert got == d - t - 1, (qi, ri, d, t, got)
                assert (got < 0) == (d <= t)
            else:
                assert got >= 1, (qi, ri, got)  # never a candidate
