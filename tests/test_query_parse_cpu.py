"""The query box of Fig. 1 (Fig. 3 step 2) is parsed on the host by the C ABI
(fps_parse_query / fps_parse_queries: no device work).  Checked against the
oracle's plain parser on typed lists and on malformed ones."""
import random

import numpy as np
import pytest

import fpsynth
import oracle
import paper_1906_06170_amd as fps


def typed(keys, width, sep=",", trailing=False, pad=""):
    first = 0 if width == 167 else 1
    vals = ["1" if j in keys else "0" for j in range(first, 167)]
    return pad + "[" + sep.join(vals) + ("," if trailing else "") + "]" + pad


def test_typed_lists_match_the_oracle():
    rnd = random.Random(3)
    for t in range(300):
        keys = set(rnd.sample(range(1, 167), rnd.randint(0, 166)))
        s = typed(keys, 166 if t % 2 else 167, [",", ", ", " ,\t"][t % 3], t % 5 == 0,
                  [" ", "", "\t\n"][t % 3])
        assert np.array_equal(fps.parse_query(s), oracle.parse_query(s)), s


def test_generated_query_text_round_trips():
    lib = fpsynth.make_library(200, 4)
    for i in range(200):
        s = fpsynth.query_text(lib.words[i], width=166 + i % 2, trailing_comma=i % 2 == 0,
                               spaces=i % 3 == 0)
        assert np.array_equal(fps.parse_query(s), lib.words[i])


BAD = ["", "[]", "[" + ",".join(["0"] * 165) + "]", "[" + ",".join(["0"] * 168) + "]",
       "[" + ",".join(["0"] * 165 + ["2"]) + "]", "[" + ",".join(["0"] * 166),
       "[" + ",".join(["0"] * 166) + "] x", "[" + ",,".join(["0"] * 166) + "]",
       "(" + ",".join(["0"] * 166) + ")", "[" + ",".join(["0"] * 166) + ",,]"]


@pytest.mark.parametrize("s", BAD, ids=range(len(BAD)))
def test_malformed_lists_rejected_by_both(s):
    with pytest.raises(ValueError):
        oracle.parse_query(s)
    with pytest.raises(fps.FPSError) as e:
        fps.parse_query(s)
    assert e.value.status == fps.FPS_E_ARG


def test_position_zero_is_a_fingerprint_error():
    s = "[1" + ",0" * 166 + "]"
    with pytest.raises(ValueError):
        oracle.parse_query(s)
    with pytest.raises(fps.FPSError) as e:
        fps.parse_query(s)
    assert e.value.status == fps.FPS_E_FINGERPRINT


def test_batch_lines_and_line_numbers():
    lib = fpsynth.make_library(20, 8)
    lines = [fpsynth.query_text(w) for w in lib.words]
    text = "\n\n".join(lines) + "\n   \n"
    assert np.array_equal(fps.parse_queries(text), oracle.parse_queries(text))
    assert np.array_equal(fps.parse_queries(text), lib.words)
    bad = lines[:5] + ["[0,1]"] + lines[5:]
    with pytest.raises(ValueError, match="line 6"):
        oracle.parse_queries("\n".join(bad))
    with pytest.raises(fps.FPSError, match="line 6"):
        fps.parse_queries("\n".join(bad))
