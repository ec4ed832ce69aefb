"""The serving loop's batch-formation policy (csrc/batcher.h), compiled by the
host compiler alone and driven through fixed scenarios: the online service-time
fit, the query cap, the deadline cap and its release when the queue is behind,
and the test that wakes reserve slots."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1906_06170_amd", "csrc")


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("batcher") / "batcher_check")
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(ROOT, "tests", "batcher_check.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return {k: float(v) for k, v in (line.split() for line in out.strip().splitlines())}


def test_fit_recovers_linear_law(results):
    assert results["fit_c0"] == pytest.approx(300.0, rel=1e-6)
    assert results["fit_c1"] == pytest.approx(4.0, rel=1e-6)


def test_fit_without_spread_is_proportional(results):
    assert results["flat_c0"] == 0.0
    assert results["flat_c1"] == pytest.approx(20.0)


def test_weight_grows_with_k(results):
    assert results["weight_q10_k700"] == pytest.approx(20.0)


def test_query_cap(results):
    assert results["cap_only"] == 3          # 3 x 10 queries <= 35 < 4 x 10
    assert results["first_over_cap"] == 1    # a request above the cap still runs alone
    assert results["empty"] == 0


def test_deadline_cap(results):
    # 300 + 40 n <= 10000 us
    assert results["deadline"] == 242
    assert results["deadline_off"] == 400
    # 5 ms already spent: 300 + 40 n <= 5000
    assert results["deadline_aged"] == 117
    # twice the weight per request
    assert results["deadline_k700"] == 121


def test_behind_queue_grows_to_query_cap(results):
    assert results["behind"] == 200          # 2000 queries / 10
    assert results["behind_mixed"] == 200


def test_deadline_request_joins_only_while_met(results):
    # a 1 ms deadline at position 30: the 30 requests ahead already take
    # 300 + 40 * 31 > 1000 us, so it starts the next batch
    assert results["late_joiner"] == 30
    # at position 10 it fits (300 + 40 * 11 = 740 us); later requests join while
    # 300 + 40 n <= 1000, i.e. n <= 17
    assert results["early_joiner"] == 17


def test_queue_behind(results):
    assert results["behind_no"] == 0
    assert results["behind_yes"] == 1
    assert results["behind_none"] == 0


def test_reserve_slots_wait_for_overload(results):
    assert results["reserve_full"] == 1      # behind, a full batch waiting
    assert results["reserve_short"] == 0     # behind, but less than a batch
    assert results["reserve_on_time"] == 0   # a full batch, but on time
