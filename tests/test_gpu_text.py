"""The library file and the query box (Fig. 3 steps 1, 2 and 5; Fig. 1) on the
GPU against the CPU oracle: the oracle reads the same text with its own
line-by-line reader, searches its own records and maps result rows to ids;
the GPU parses the text in HBM, searches and maps rows to ids through the C
ABI.  Ids, distances, order and the first malformed line must agree exactly."""
import numpy as np
import pytest

import fpsynth
import oracle

fps = pytest.importorskip("paper_1906_06170_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def oracle_ids(words, ids, query, k, ranges=None):
    h = oracle.search(words, query, k, ranges=ranges)
    return ids[h["index"]], h["distance"]


FORMATS = [(167, " ", False, True), (166, "\t", True, True), (167, ",", False, False),
           (166, " " * 40, True, False)]


@pytest.mark.parametrize("fmt", FORMATS, ids=["167-space", "166-tab-crlf", "167-comma-noeol",
                                              "166-wide-sep-crlf-noeol"])
@pytest.mark.parametrize("n", [1, 7, 1000, 100_000])
def test_text_library_matches_oracle(n, fmt):
    width, sep, crlf, final = fmt
    say("case: text library n", n, "format", fmt)
    lib_np = fpsynth.make_library(n, 3 + n % 5)
    ids = fpsynth.make_cids(n, 11)
    text = fpsynth.library_text(lib_np.words, ids, width=width, sep=sep, crlf=crlf,
                                final_eol=final)
    owords, oids = oracle.read_text(text)
    cut = [0, n // 3, n // 2, n] if n >= 4 else None
    lib = fps.Library(text=text, strides=cut)
    assert lib.n == len(owords)
    assert np.array_equal(lib.ids, oids)
    qs = fpsynth.batch_queries(lib_np, 6, 500 + n).words
    for qi in range(len(qs)):
        for k, mask in ((30, fps.MASK_ALL), (1, 1), (1000, 6 if cut else fps.MASK_ALL)):
            got = lib.search_ids(qs[qi], k, mask)
            rr = None if mask == fps.MASK_ALL else oracle.mask_ranges(cut or [0, n], mask)
            wid, wd = oracle_ids(owords, oids, qs[qi], k, rr)
            assert np.array_equal(got["id"], wid), (qi, k, mask)
            assert np.array_equal(got["distance"], wd), (qi, k, mask)
    # the parsed library equals one uploaded from the words (same device bytes)
    ref = fps.Library(owords, strides=cut)
    assert torch.equal(lib._buf, ref._buf)
    lib.close()
    ref.close()


def malformed(line: str, n=40_000, at=(1, 17_123, 40_000), seed=5):
    """Texts of n lines with one malformed line at each position in `at`."""
    lib_np = fpsynth.make_library(n, seed)
    ids = fpsynth.make_cids(n, 1)
    good = fpsynth.library_text(lib_np.words, ids).tobytes().split(b"\n")[:-1]
    for a in at:
        lines = list(good)
        lines[a - 1] = line.encode()
        yield a, b"\n".join(lines) + b"\n"


BAD_LINES = {
    1: "5 " + "0" * 167 + " " * 100,
    2: "",
    3: "5x" + "0" * 167,
    4: "5 " + "0" * 100 + "2" + "0" * 66,
    5: "5 1" + "0" * 166,
    6: "5 " + "0" * 167 + " #",
}
EXTRA = {2: ["  5 " + "0" * 167, "1" * 20 + " " + "0" * 167, "\r"],
         4: ["5 " + "0" * 168, "5 " + "0" * 165]}


@pytest.mark.parametrize("kind", sorted(BAD_LINES))
def test_malformed_line_reported_like_the_oracle(kind):
    for line in [BAD_LINES[kind]] + EXTRA.get(kind, []):
        for at, text in malformed(line):
            say("case: malformed kind", kind, "line", at, repr(line[:12]))
            with pytest.raises(oracle.TextError) as oe:
                oracle.read_text(text)
            assert (oe.value.line, oe.value.kind) == (at, kind)
            with pytest.raises(fps.FPSError) as ge:
                fps.Library(text=text)
            want = fps.FPS_E_FINGERPRINT if kind == 5 else fps.FPS_E_ARG
            assert ge.value.status == want
            assert f"line {at}:" in str(ge.value), str(ge.value)


def test_first_malformed_line_wins():
    lines = [BAD_LINES[6], BAD_LINES[3]]
    for at, text in malformed(lines[0], at=(30_001,)):
        t = text.split(b"\n")
        t[9_999] = lines[1].encode()
        text = b"\n".join(t)
        with pytest.raises(oracle.TextError) as oe:
            oracle.read_text(text)
        with pytest.raises(fps.FPSError) as ge:
            fps.Library(text=text)
        assert (oe.value.line, oe.value.kind) == (10_000, 3)
        assert "line 10000:" in str(ge.value)


def test_text_edge_cases():
    # hand-typed lines: short and 19-digit ids, leading zeros, mixed widths, blanks
    keys = [{1}, {166}, set(range(1, 167)), set()]
    lines = []
    for i, ks in enumerate(keys):
        width = 167 if i % 2 else 166
        first = 0 if width == 167 else 1
        ident = ["7", "9999999999999999999", "000123", "42"][i]
        lines.append(ident + [" ", "\t\t", " , ", ","][i]
                     + "".join("1" if j in ks else "0" for j in range(first, 167))
                     + ["", "\r", "  ", "\t"][i])
    for final in ("", "\n"):
        text = "\n".join(lines) + final
        owords, oids = oracle.read_text(text)
        lib = fps.Library(text=text.encode())
        assert lib.n == 4 and np.array_equal(lib.ids, oids)
        assert oids.tolist() == [7, 9999999999999999999, 123, 42]
        for q in range(4):
            got = lib.search_ids(owords[q], 4)
            wid, wd = oracle_ids(owords, oids, owords[q], 4)
            assert np.array_equal(got["id"], wid) and np.array_equal(got["distance"], wd)
        lib.close()
    # empty line at the end of the text only: one record; an empty text: error
    with pytest.raises(fps.FPSError):
        fps.Library(text=b"\n")
    with pytest.raises(fps.FPSError):
        fps.Library(text=(lines[0] + "\n\n").encode())
    with pytest.raises((fps.FPSError, ValueError)):
        fps.Library(text=b"")


def test_query_box_search_matches_oracle():
    """A target typed as the bracketed list of Fig. 1, results as (CID,
    distance) pairs in ascending order (Fig. 2)."""
    n = 50_000
    lib_np = fpsynth.make_library(n, 9)
    ids = fpsynth.make_cids(n, 2)
    text = fpsynth.library_text(lib_np.words, ids)
    owords, oids = oracle.read_text(text)
    lib = fps.Library(text=text)
    qs = fpsynth.make_queries(lib_np, 5, 77, flips=(0, 4))
    for qi in range(5):
        typed = fpsynth.query_text(qs.words[qi], width=166 if qi % 2 else 167,
                                   trailing_comma=qi % 3 == 0, spaces=qi == 4)
        got = lib.search_ids(typed, 30)
        wid, wd = oracle_ids(owords, oids, oracle.parse_query(typed), 30)
        assert np.array_equal(got["id"], wid) and np.array_equal(got["distance"], wd)
        assert got["distance"][0] <= qs.flips[qi]
    # a batch typed one list per line, searched together
    typed = "\n".join(fpsynth.query_text(q) for q in qs.words)
    batch = fps.parse_queries(typed)
    assert np.array_equal(batch, oracle.parse_queries(typed))
    hits, off = lib.search_batch(batch, 30)
    for qi in range(5):
        h = hits[int(off[qi]):int(off[qi + 1])]
        wid, wd = oracle_ids(owords, oids, batch[qi], 30)
        assert np.array_equal(lib.hit_ids(h), wid) and np.array_equal(h["distance"], wd)
    lib.close()


def test_hit_ids_without_id_table_is_refused():
    lib_np = fpsynth.make_library(100, 1)
    lib = fps.Library(lib_np.words)
    h = lib.search(lib_np.words[0], 3)
    with pytest.raises(fps.FPSError) as e:
        lib.hit_ids(h)
    assert e.value.status == fps.FPS_E_STATE


def test_device_only_ids_match_oracle():
    """A text library whose id column stays in device memory (host_ids=False):
    the ids of every hit are gathered on the device and equal the oracle's, for
    single queries, a batch of 40 (about 40,000 hits, staging grown on demand)
    and an empty hit list; an index beyond the library is refused first."""
    n = 100_000
    lib_np = fpsynth.make_library(n, 13)
    ids = fpsynth.make_cids(n, 14)
    text = fpsynth.library_text(lib_np.words, ids)
    owords, oids = oracle.read_text(text)
    lib = fps.Library(text=text, host_ids=False)
    assert lib.ids is None
    assert np.array_equal(lib.ids_device.cpu().numpy().astype(np.uint64), oids)
    qs = fpsynth.batch_queries(lib_np, 40, 15).words
    for qi in range(3):
        got = lib.search_ids(qs[qi], 30)
        wid, wd = oracle_ids(owords, oids, qs[qi], 30)
        assert np.array_equal(got["id"], wid) and np.array_equal(got["distance"], wd)
    hits, off = lib.search_batch(qs, 1000)
    got = lib.hit_ids(hits)
    assert np.array_equal(got, oids[hits["index"]])
    assert len(lib.hit_ids(hits[:0])) == 0
    bad = hits[:2].copy()
    bad["index"][1] = n
    with pytest.raises(fps.FPSError) as e:
        lib.hit_ids(bad)
    assert e.value.status == fps.FPS_E_ARG
    lib.close()


def test_counts_reused_and_changed_text_detected():
    """fps_text_library_load reuses the counts fps_text_count left in the
    workspace for the same text; a text whose lines moved across a chunk
    boundary between the two calls is refused ("the text changed since it was
    counted") instead of being parsed into wrong rows; counted again, the same
    text gets the ordinary validation (its split line is malformed)."""
    import ctypes
    n = 40_000
    lib_np = fpsynth.make_library(n, 21)
    ids = fpsynth.make_cids(n, 22)
    text = fpsynth.library_text(lib_np.words, ids)
    c = fps.load_library()
    dtext = torch.from_numpy(np.frombuffer(bytes(text), dtype=np.uint8).copy()).to("cuda")
    nt = int(dtext.numel())
    wsb = ctypes.c_size_t()
    assert c.fps_text_workspace_bytes(nt, ctypes.byref(wsb)) == fps.FPS_OK
    tws = torch.empty(int(wsb.value), dtype=torch.uint8, device="cuda")
    cnt = ctypes.c_uint64()

    def count():
        assert c.fps_text_count(ctypes.c_void_p(dtext.data_ptr()), nt,
                                ctypes.c_void_p(tws.data_ptr()), tws.numel(), None,
                                ctypes.byref(cnt)) == fps.FPS_OK
        return int(cnt.value)

    def load(nrec):
        nbytes = int(c.fps_library_device_bytes(nrec))
        buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        idd = torch.empty(nrec, dtype=torch.int64, device="cuda")
        h = ctypes.c_void_p()
        rc = c.fps_text_library_load(ctypes.c_void_p(dtext.data_ptr()), nt, nrec, None, 0,
                                     ctypes.c_void_p(tws.data_ptr()), tws.numel(),
                                     ctypes.c_void_p(buf.data_ptr()), nbytes,
                                     ctypes.c_void_p(idd.data_ptr()), None, None, ctypes.byref(h))
        msg = c.fps_last_error().decode() if rc else ""
        if rc == fps.FPS_OK:
            c.fps_library_free(h)
        return rc, msg, buf, idd

    assert count() == n
    rc, _, buf, idd = load(n)
    assert rc == fps.FPS_OK
    assert np.array_equal(idd.cpu().numpy().astype(np.uint64), ids)
    ref = fps.Library(lib_np.words)
    assert torch.equal(buf, ref._buf)
    ref.close()
    # the line that straddles the boundary of chunks 99 and 100 (16,384 bytes
    # each) ends one character after its id instead: its newline moves into
    # chunk 99, the line count stays n
    host = dtext.cpu().numpy()
    nls = np.nonzero(host == 10)[0]
    boundary = 100 * 16384
    L = int(np.searchsorted(nls, boundary))  # first newline at or past the boundary
    start = int(nls[L - 1]) + 1
    sep = start + int(np.nonzero(host[start:nls[L]] == 32)[0][0])
    assert sep < boundary <= int(nls[L])
    host[int(nls[L])] = 32
    host[sep] = 10
    dtext.copy_(torch.from_numpy(host).to("cuda"))
    rc, msg, _, _ = load(n)
    say("changed text:", msg)
    assert rc == fps.FPS_E_ARG and "changed since it was counted" in msg
    assert count() == n
    rc, msg, _, _ = load(n)
    say("counted again:", msg)
    assert rc == fps.FPS_E_ARG and "changed" not in msg and msg.startswith("line ")
