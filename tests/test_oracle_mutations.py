"""Plants plausible mistakes in copies of the oracle's C source (on the CPU) and
checks that the pins catch every one of them.  Each mutated build runs in its own
process, so a mistake that corrupts memory cannot take the test runner down."""
import json
import os
import subprocess
import sys

import pytest

import oracle

MUTATIONS = {
    "drop_last_key": ("j <= ORACLE_KEYS", "j < ORACLE_KEYS"),
    "drop_first_key": ("for (int j = 1; j <= ORACLE_KEYS", "for (int j = 2; j <= ORACLE_KEYS"),
    "no_abs": ("sum += (c < 0) ? -c : c;", "sum += c;"),
    "same_operand": ("key_value(a, j) - key_value(b, j)", "key_value(a, j) - key_value(a, j)"),
    "wrong_word": ("rec[j >> 6] >> (j & 63)", "rec[j >> 7] >> (j & 63)"),
    "ties_descending": ("(d0 == d1 && i0 < i1)", "(d0 == d1 && i0 > i1)"),
    "ties_ignored": ("d0 < d1 || (d0 == d1 && i0 < i1)", "d0 < d1"),
    "keep_largest": ("return d0 < d1 ||", "return d0 > d1 ||"),
    "k_minus_one": ("uint64_t want = k < total ? k : total;",
                    "uint64_t want = k < total ? (k ? k - 1 : 0) : total;"),
    "merge_drops_chunk": ("for (int j = 0; j < njobs; ++j)\n      for",
                          "for (int j = 1; j < njobs; ++j)\n      for"),
    "range_end_skipped": ("for (uint64_t i = begin[r]; i < end[r]; ++i)\n      topk_offer",
                          "for (uint64_t i = begin[r]; i + 1 < end[r]; ++i)\n      topk_offer"),
    # the library-file reader (Fig. 3 step 1)
    "text_key_offset": ("uint64_t first_key = (width == 167) ? 0 : 1;", "uint64_t first_key = 1;"),
    "text_long_ids": ("if (p == 0 || p > 19) return 2;", "if (p == 0) return 2;"),
    "text_tail_unchecked": ("if (!is_blank(s[t])) return 6;", "if (s[t] == 0) return 6;"),
    "text_no_cr": ("c == ' ' || c == '\\t' || c == '\\r'; }", "c == ' ' || c == '\\t'; }"),
    "text_key0_unchecked": ("if (j == 0) return 5;", "if (j == 0) j = 0;"),
    # wider fingerprints (Section 5, remark 3)
    "wide_drop_last_key": ("j < 64 * words; ++j", "j < 64 * words - 1; ++j"),
    "wide_wrong_word": ("rec[j >> 6] >> (j & 63)) & 1u);\n}\n\nuint32_t oracle_distance_w",
                        "rec[j >> 7] >> (j & 63)) & 1u);\n}\n\nuint32_t oracle_distance_w"),
    "wide_record_stride": ("topk_offer(t, (uint32_t)i, oracle_distance_w(lib + (uint64_t)words * i",
                           "topk_offer(t, (uint32_t)i, oracle_distance_w(lib + (uint64_t)3 * i"),
}

RUNNER = r"""
import json, sys
sys.path.insert(0, sys.argv[2]); sys.path.insert(0, sys.argv[3])
import oracle
from pins import ALL_PINS
orc = oracle.Oracle(sys.argv[1])
failed = []
for pin in ALL_PINS:
    try:
        pin(orc)
    except AssertionError:
        failed.append(pin.__name__)
    print(json.dumps({"pin": pin.__name__, "failed": failed}), flush=True)
"""


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(oracle.SOURCE).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    cpath = os.path.join(tmp_path, "oracle_mut.c")
    with open(cpath, "w") as f:
        f.write(src.replace(old, new, 1))
    so = oracle.compile_source(cpath, os.path.join(tmp_path, "oracle_mut.so"))
    here = os.path.dirname(os.path.abspath(__file__))
    root = os.path.dirname(here)
    p = subprocess.run([sys.executable, "-c", RUNNER, so, here, root], capture_output=True,
                       text=True, timeout=600)
    lines = [json.loads(x) for x in p.stdout.splitlines() if x.startswith("{")]
    failed = lines[-1]["failed"] if lines else []
    crashed = p.returncode != 0
    assert failed or crashed, f"no pin catches the planted mistake {name}"
