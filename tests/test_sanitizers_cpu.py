"""Host code under the sanitizers: the CPU oracle and the input generator
(tests/sanitize_check.c, against a brute force of its own) and the serving
loop's batching policy (tests/batcher_check.cpp), built by the host compilers
with AddressSanitizer + UndefinedBehaviorSanitizer, and the oracle's threaded
form with ThreadSanitizer.  No device code is built here."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C_SRC = [os.path.join(ROOT, "tests", "sanitize_check.c"), os.path.join(ROOT, "oracle", "oracle.c"),
         os.path.join(ROOT, "fpsynth", "gen.c")]
ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
TSAN = ["-fsanitize=thread"]


def _build_run(tmp_path, compiler, std, flags, sources, name):
    cc = shutil.which(compiler)
    if cc is None:
        pytest.skip(f"no {compiler}")
    exe = str(tmp_path / name)
    try:
        subprocess.run([cc, std, "-O1", "-g", *flags, "-pthread", "-I",
                        os.path.join(ROOT, "paper_1906_06170_amd", "csrc"), *sources, "-o", exe],
                       check=True, capture_output=True, text=True)
    except subprocess.CalledProcessError as e:
        if "sanitize" in e.stderr and ("cannot find" in e.stderr or "unrecognized" in e.stderr):
            pytest.skip(f"sanitizer runtime unavailable: {e.stderr[:200]}")
        raise
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return r.stdout


def test_oracle_and_generator_asan_ubsan(tmp_path):
    assert _build_run(tmp_path, "gcc", "-std=c11", ASAN, C_SRC, "san_c").strip() == "ok"


def test_oracle_threads_tsan(tmp_path):
    assert _build_run(tmp_path, "gcc", "-std=c11", TSAN, C_SRC, "tsan_c").strip() == "ok"


def test_batcher_asan_ubsan(tmp_path):
    out = _build_run(tmp_path, "g++", "-std=c++17", ASAN,
                     [os.path.join(ROOT, "tests", "batcher_check.cpp")], "san_batcher")
    assert "fit_c1" in out and "behind_yes 1" in out
