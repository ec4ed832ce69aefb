"""Python binding of libfps.so, the MI355X exact fingerprint top-k engine.

Argument marshalling only: every step of a search runs in the HIP library
(include/fps.h).  PyTorch supplies device memory (the library rows and the
workspaces are torch tensors owned by the objects below) and the current HIP
stream.  There is no CPU path: importing the binding without a built
libfps.so raises, and so does using it without a GPU.

The problem is the one of FPScreen (arXiv 1906.06170), Fig. 3: the N library
records nearest to a MACCS-166 query under the Manhattan distance of Section
4.3, ascending, ties by library index; searches may be restricted to strides
of the library (Section 2.1) and merged globally (Section 4.3).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "libfps.so")

FPS_OK, FPS_E_ARG, FPS_E_FINGERPRINT, FPS_E_NOMEM, FPS_E_DEVICE, FPS_E_STATE, FPS_E_BUSY = (
    0, -1, -2, -3, -4, -5, -6)
STATUS_NAMES = {0: "FPS_OK", -1: "FPS_E_ARG", -2: "FPS_E_FINGERPRINT", -3: "FPS_E_NOMEM",
                -4: "FPS_E_DEVICE", -5: "FPS_E_STATE", -6: "FPS_E_BUSY"}
MASK_ALL = 0xFFFFFFFF
PATH_AUTO, PATH_SINGLE, PATH_POPCOUNT, PATH_MFMA_I8, PATH_MFMA_F4 = 0, 1, 2, 3, 4
PATH_NAMES = {0: "auto", 1: "single", 2: "popcount", 3: "mfma_i8", 4: "mfma_f4"}

HIT_DTYPE = np.dtype([("index", np.uint32), ("distance", np.uint32)])


class FPSError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class SearchStats(ctypes.Structure):
    _fields_ = [("path", ctypes.c_uint32), ("queries", ctypes.c_uint32),
                ("fallbacks", ctypes.c_uint32), ("variant", ctypes.c_uint32),
                ("candidates", ctypes.c_uint64), ("scan_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("graph", ctypes.c_uint32),
                ("scan_launches", ctypes.c_uint32), ("scan_ms_sum", ctypes.c_double),
                ("total_ms_sum", ctypes.c_double), ("calls", ctypes.c_uint64),
                ("scan_launches_sum", ctypes.c_uint64)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_size_t), ("max_batch_queries", ctypes.c_uint32),
                ("max_wait_us", ctypes.c_uint32), ("n_streams", ctypes.c_uint32),
                ("deadline_cap", ctypes.c_uint32), ("reserve_streams", ctypes.c_uint32),
                ("tune_k", ctypes.c_void_p), ("n_tune_k", ctypes.c_uint32)]


class RequestStats(ctypes.Structure):
    _fields_ = [("arrival_ns", ctypes.c_uint64), ("submit_ns", ctypes.c_uint64),
                ("start_ns", ctypes.c_uint64), ("done_ns", ctypes.c_uint64),
                ("batch_id", ctypes.c_uint32), ("batch_queries", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_uint64), ("queries", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("deadline_misses", ctypes.c_uint64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("max_us", ctypes.c_double), ("mean_batch_queries", ctypes.c_double),
                ("cost_fixed_us", ctypes.c_double), ("cost_per_weight_us", ctypes.c_double),
                ("admit_p50_us", ctypes.c_double), ("admit_p99_us", ctypes.c_double),
                ("untuned_batches", ctypes.c_uint64)]


CLUSTER_MAX_K = 16
CLUSTER_MAX_Q = 16384


class ClusterInfo(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("rounds", ctypes.c_uint32),
                ("score", ctypes.c_double * (CLUSTER_MAX_K + 1))]


def _cluster_result(info, labels, centers, k_min, k_max):
    return {"K": int(info.k), "labels": labels.astype(np.int64), "rounds": int(info.rounds),
            "centers": centers[:info.k].copy(),
            "scores": {K: float(info.score[K]) for K in range(k_min, k_max + 1)}}


EXPORTS = {
    # name: (restype, argtypes)
    "fps_library_device_bytes": (ctypes.c_size_t, [ctypes.c_uint64]),
    "fps_library_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                        ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "fps_library_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "fps_library_free": (ctypes.c_int, [ctypes.c_void_p]),
    "fps_set_path": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "fps_set_variant": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "fps_set_graphs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "fps_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "fps_workspace_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "fps_search": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                  ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fps_search_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "fps_search_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_size_t, ctypes.c_void_p, ctypes.c_uint64,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "fps_last_search_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fps_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                ctypes.c_void_p]),
    "fps_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_uint64,
                                      ctypes.c_uint64, ctypes.c_int]),
    "fps_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_size_t, ctypes.c_void_p]),
    "fps_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                         ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]),
    "fps_server_result_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64,
                                              ctypes.c_void_p, ctypes.c_void_p]),
    "fps_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                       ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64,
                                       ctypes.c_void_p]),
    "fps_server_stats_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "fps_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "fps_clock_ns": (ctypes.c_uint64, []),
    "fps_text_workspace_bytes": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_void_p]),
    "fps_text_count": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                      ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]),
    "fps_text_library_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                             ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                             ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "fps_hit_ids": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                   ctypes.c_void_p]),
    "fps_parse_query": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t, ctypes.c_void_p]),
    "fps_parse_queries": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t, ctypes.c_void_p,
                                         ctypes.c_uint32, ctypes.c_void_p]),
    "fps_wide_device_bytes": (ctypes.c_size_t, [ctypes.c_uint64, ctypes.c_uint32]),
    "fps_wide_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                     ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]),
    "fps_wide_free": (ctypes.c_int, [ctypes.c_void_p]),
    "fps_wide_set_path": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "fps_wide_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_uint64,
                                           ctypes.c_int]),
    "fps_wide_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "fps_wide_workspace_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32,
                                                ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p]),
    "fps_wide_search_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_size_t, ctypes.c_void_p, ctypes.c_uint64,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "fps_wide_search": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fps_wide_last_search_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fps_cluster_workspace_bytes": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_void_p]),
    "fps_cluster": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                   ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "fps_cluster_search_workspace_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32,
                                                          ctypes.c_uint32, ctypes.c_uint32,
                                                          ctypes.c_uint32, ctypes.c_void_p]),
    "fps_cluster_search": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p, ctypes.c_uint64,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "fps_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load_library(path: str = SO_PATH):
    """ctypes handle of libfps.so with argument types set.  Raises if not built."""
    global _lib
    if _lib is not None and path == SO_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path == SO_PATH:
        _lib = lib
    return lib


def _check(rc: int):
    if rc != FPS_OK:
        msg = load_library().fps_last_error()
        raise FPSError(rc, msg.decode() if msg else "")


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _stream(stream, device: int | None = None):
    """HIP stream handle: the given torch stream, else torch's current stream
    on `device` (the raw-stream query is the cheap form of current_stream())."""
    import torch
    if stream is not None:
        return ctypes.c_void_p(stream.cuda_stream)
    if device is not None and hasattr(torch._C, "_cuda_getCurrentRawStream"):
        return ctypes.c_void_p(torch._C._cuda_getCurrentRawStream(device))
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the fingerprint engine needs a ROCm GPU; none is visible")
    return torch


def device_bytes(n: int) -> int:
    return int(load_library().fps_library_device_bytes(n))


def _u32(a, n, default=None) -> np.ndarray:
    if a is None:
        return np.full(n, default, dtype=np.uint32)
    a = np.asarray(a)
    if a.ndim == 0:
        return np.full(n, int(a), dtype=np.uint32)
    return np.ascontiguousarray(a, dtype=np.uint32)


ID_HIT_DTYPE = np.dtype([("id", np.uint64), ("distance", np.uint32)])


def parse_query(text: str) -> np.ndarray:
    """The target as typed into the search box of Fig. 1 ("[0,1,...,0,]"):
    the three fingerprint words (fps_parse_query)."""
    b = text.encode() if isinstance(text, str) else bytes(text)
    out = np.zeros(3, dtype=np.uint64)
    _check(load_library().fps_parse_query(b, len(b), _ptr(out)))
    return out


def parse_queries(text: str) -> np.ndarray:
    """One bracketed list per line (blank lines skipped): (q, 3) words."""
    b = text.encode() if isinstance(text, str) else bytes(text)
    cap = b.count(b"\n") + 1
    out = np.zeros((cap, 3), dtype=np.uint64)
    nq = ctypes.c_uint32()
    _check(load_library().fps_parse_queries(b, len(b), _ptr(out), cap, ctypes.byref(nq)))
    return out[:nq.value].copy()


class Library:
    """A fingerprint library resident in HBM (Fig. 3 step 1).

    Library(words) uploads (n, 3) fingerprint words; Library(text=...) parses a
    library file (bytes, a uint8 array, or a uint8 torch tensor already on the
    GPU) on the GPU and keeps its id column: in device memory (Library.ids_device)
    and, with host_ids=True (the default), also on the host (Library.ids)."""

    def __init__(self, words: np.ndarray | None = None, strides=None, stream=None, *,
                 text=None, host_ids: bool = True):
        torch = _require_gpu()
        c = load_library()
        self._ws = None
        self._ws_sizes = {}
        self._handle = ctypes.c_void_p()
        self.ids = None
        self.text_stats = None
        if (words is None) == (text is None):
            raise ValueError("give either words or text")
        if text is not None:
            self._load_text(torch, c, text, strides, stream, host_ids)
            return
        w = np.ascontiguousarray(words, dtype=np.uint64).reshape(-1, 3)
        self.n = int(w.shape[0])
        nbytes = int(c.fps_library_device_bytes(self.n))
        self._buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self._device = self._buf.device.index
        st, ns = self._stride_table(strides)
        _check(c.fps_library_load(_ptr(w), self.n, None if st is None else _ptr(st), ns,
                                  ctypes.c_void_p(self._buf.data_ptr()), nbytes, _stream(stream),
                                  ctypes.byref(self._handle)))

    def _stride_table(self, strides):
        self.strides = [0, self.n] if strides is None else [int(x) for x in strides]
        if strides is None:
            return None, 0
        st = np.ascontiguousarray(strides, dtype=np.uint64)
        return st, len(st) - 1

    def _load_text(self, torch, c, text, strides, stream, host_ids):
        if isinstance(text, torch.Tensor):
            dtext = text if text.is_cuda else text.to("cuda")
        else:
            if isinstance(text, (bytes, bytearray, memoryview)):
                text = np.frombuffer(bytes(text), dtype=np.uint8)
            text = np.ascontiguousarray(text, dtype=np.uint8).reshape(-1)
            if not text.flags.writeable:
                text = text.copy()
            dtext = torch.from_numpy(text).to("cuda")
        dtext = dtext.contiguous()
        nt = int(dtext.numel())
        wsb = ctypes.c_size_t()
        _check(c.fps_text_workspace_bytes(nt, ctypes.byref(wsb)))
        tws = torch.empty(max(int(wsb.value), 256), dtype=torch.uint8, device="cuda")
        n = ctypes.c_uint64()
        s = _stream(stream)
        _check(c.fps_text_count(ctypes.c_void_p(dtext.data_ptr()), nt,
                                ctypes.c_void_p(tws.data_ptr()), tws.numel(), s,
                                ctypes.byref(n)))
        self.n = int(n.value)
        nbytes = int(c.fps_library_device_bytes(self.n))
        self._buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self._device = self._buf.device.index
        self._ids_dev = torch.empty(max(self.n, 1), dtype=torch.int64, device="cuda")
        self.ids = np.empty(max(self.n, 1), dtype=np.uint64) if host_ids else None
        st, ns = self._stride_table(strides)
        _check(c.fps_text_library_load(
            ctypes.c_void_p(dtext.data_ptr()), nt, self.n, None if st is None else _ptr(st), ns,
            ctypes.c_void_p(tws.data_ptr()), tws.numel(), ctypes.c_void_p(self._buf.data_ptr()),
            nbytes, ctypes.c_void_p(self._ids_dev.data_ptr()),
            _ptr(self.ids) if host_ids else None, s, ctypes.byref(self._handle)))
        if host_ids:
            self.ids = self.ids[:self.n]

    @property
    def ids_device(self):
        """The id column in device memory (int64 tensor of n; ids are below 2^63 only
        when they fit 19 digits, which every valid id does), or None."""
        ids = getattr(self, "_ids_dev", None)
        return None if ids is None else ids[:self.n]

    # -- helpers --------------------------------------------------------------
    @property
    def handle(self):
        return self._handle

    def close(self):
        if self._handle:
            load_library().fps_library_free(self._handle)
            self._handle = ctypes.c_void_p()
        self._buf = None
        self._ws = None
        self._ids_dev = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, k, mask=None, q: int | None = None) -> int:
        k = np.atleast_1d(np.asarray(k))
        q = len(k) if q is None else q
        kk = _u32(k if len(k) == q else np.full(q, int(k[0])), q)
        mm = None if mask is None else _u32(mask, q)
        out = ctypes.c_size_t()
        _check(load_library().fps_workspace_bytes(self._handle, q, _ptr(kk),
                                                  None if mm is None else _ptr(mm),
                                                  ctypes.byref(out)))
        return int(out.value)

    def _workspace(self, nbytes: int):
        import torch
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device="cuda")
        return self._ws

    def set_path(self, path: int):
        _check(load_library().fps_set_path(self._handle, int(path)))

    def set_graphs(self, enable: bool):
        """Replay repeated launch shapes from HIP graphs (default on)."""
        _check(load_library().fps_set_graphs(self._handle, int(bool(enable))))

    def set_timing(self, enable: bool):
        """Device timing (scan_ms, total_ms in last_stats) with HIP events;
        off by default, since the events lengthen a single-query search."""
        _check(load_library().fps_set_timing(self._handle, int(bool(enable))))

    def set_variant(self, variant: int):
        """Matrix-core tile shape (0..3, or -1 for the tuner's choice)."""
        _check(load_library().fps_set_variant(self._handle, int(variant)))

    def set_tuning(self, candidate_scale: float = 1.0, sample_records: int = 0,
                   phase_records: int = 0, force_fallback: bool = False):
        """Capacity / bound-sample / phase knobs (results never depend on them)."""
        self._ws_sizes = {}
        _check(load_library().fps_set_tuning(self._handle, float(candidate_scale),
                                             int(sample_records), int(phase_records),
                                             int(bool(force_fallback))))

    def last_stats(self) -> dict:
        st = SearchStats()
        _check(load_library().fps_last_search_stats(self._handle, ctypes.byref(st)))
        return {"path": PATH_NAMES.get(st.path, st.path), "queries": st.queries,
                "fallbacks": st.fallbacks, "candidates": st.candidates, "variant": st.variant,
                "scan_ms": st.scan_ms, "total_ms": st.total_ms, "graph": bool(st.graph),
                "scan_launches": st.scan_launches, "scan_ms_sum": st.scan_ms_sum,
                "total_ms_sum": st.total_ms_sum, "calls": st.calls,
                "scan_launches_sum": st.scan_launches_sum}

    def tune(self, nq: int, k, mask=None, stream=None):
        """Runs the autotuner for a batch shape of nq queries ahead of use."""
        kk = _u32(k, nq)
        mm = None if mask is None else _u32(mask, nq)
        nb = ctypes.c_size_t()
        _check(load_library().fps_workspace_bytes(self._handle, nq, _ptr(kk),
                                                  None if mm is None else _ptr(mm),
                                                  ctypes.byref(nb)))
        ws = self._workspace(int(nb.value))
        _check(load_library().fps_tune(self._handle, nq, _ptr(kk),
                                       None if mm is None else _ptr(mm),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                       _stream(stream, self._device)))

    # -- search ---------------------------------------------------------------
    def search(self, query, k: int, mask: int = MASK_ALL, stream=None) -> np.ndarray:
        """Top-k of one query: structured array (index, distance), ascending."""
        q = np.ascontiguousarray(np.asarray(query, dtype=np.uint64).reshape(3))
        key = (int(k), int(mask))
        nb = self._ws_sizes.get(key)
        if nb is None:
            kk = np.array([k], dtype=np.uint32)
            mm = np.array([mask], dtype=np.uint32)
            c = ctypes.c_size_t()
            _check(load_library().fps_workspace_bytes(self._handle, 1, _ptr(kk), _ptr(mm),
                                                      ctypes.byref(c)))
            nb = self._ws_sizes[key] = int(c.value)
        ws = self._workspace(nb)
        out = np.empty(max(int(k), 1), dtype=HIT_DTYPE)
        nout = ctypes.c_uint32()
        _check(load_library().fps_search(self._handle, _ptr(q), int(k), int(mask),
                                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), _ptr(out),
                                         ctypes.byref(nout), _stream(stream, self._device)))
        return out[:nout.value].copy()

    def hit_ids(self, hits: np.ndarray) -> np.ndarray:
        """Fig. 3 step 5: the id of every hit's record (libraries loaded from text)."""
        h = np.ascontiguousarray(hits, dtype=HIT_DTYPE)
        out = np.empty(max(len(h), 1), dtype=np.uint64)
        _check(load_library().fps_hit_ids(self._handle, _ptr(h), len(h), _ptr(out)))
        return out[:len(h)].copy()

    def search_ids(self, query, k: int, mask: int = MASK_ALL, stream=None) -> np.ndarray:
        """Top-k of one query as (id, distance) pairs, ascending (Fig. 2); the
        query may be given as the typed bracketed list of Fig. 1."""
        if isinstance(query, (str, bytes)):
            query = parse_query(query)
        h = self.search(query, k, mask, stream)
        out = np.empty(len(h), dtype=ID_HIT_DTYPE)
        out["id"] = self.hit_ids(h)
        out["distance"] = h["distance"]
        return out

    def cluster_search(self, queries, k: int = 30, k_min: int = 2, k_max: int = 8,
                       mask: int = MASK_ALL, max_iter: int = 100, stream=None) -> dict:
        """Batch clustering search (Section 4.4): the clustering of cluster()
        plus hits[c], the top-k of every chosen center c (fps_cluster_search)."""
        c = load_library()
        qs = np.ascontiguousarray(np.asarray(queries, dtype=np.uint64).reshape(-1, 3))
        nq = qs.shape[0]
        nb = ctypes.c_size_t()
        _check(c.fps_cluster_search_workspace_bytes(self._handle, nq, int(k_max), int(k),
                                                    int(mask), ctypes.byref(nb)))
        ws = self._workspace(int(nb.value))
        cap = max(1, int(k) * int(k_max))
        out = np.empty(cap, dtype=HIT_DTYPE)
        off = np.zeros(int(k_max) + 1, dtype=np.uint64)
        labels = np.zeros(nq, dtype=np.uint32)
        centers = np.zeros((max(k_max, 1), 3), dtype=np.uint64)
        info = ClusterInfo()
        _check(c.fps_cluster_search(self._handle, _ptr(qs), nq, int(k_min), int(k_max),
                                    int(max_iter), int(k), int(mask),
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), _ptr(out), cap,
                                    _ptr(off), _ptr(labels), _ptr(centers), ctypes.byref(info),
                                    _stream(stream, self._device)))
        res = _cluster_result(info, labels, centers, k_min, k_max)
        res["hits"] = [out[int(off[i]):int(off[i + 1])].copy() for i in range(res["K"])]
        return res

    def search_batch(self, queries, k, mask=None, stream=None):
        """Independent top-k per query.  Returns (hits, offsets): query i's hits
        are hits[offsets[i]:offsets[i+1]]."""
        qs = np.ascontiguousarray(np.asarray(queries, dtype=np.uint64).reshape(-1, 3))
        nq = qs.shape[0]
        kk = _u32(k, nq)
        mm = None if mask is None else _u32(mask, nq)
        nb = ctypes.c_size_t()
        _check(load_library().fps_workspace_bytes(self._handle, nq, _ptr(kk),
                                                  None if mm is None else _ptr(mm),
                                                  ctypes.byref(nb)))
        ws = self._workspace(int(nb.value))
        cap = int(kk.astype(np.uint64).sum())
        out = np.empty(max(cap, 1), dtype=HIT_DTYPE)
        off = np.zeros(nq + 1, dtype=np.uint64)
        _check(load_library().fps_search_batch(
            self._handle, _ptr(qs), nq, _ptr(kk), None if mm is None else _ptr(mm),
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _ptr(out), cap, _ptr(off),
            _stream(stream, self._device)))
        # a view (no second copy of up to sum(k) hits); it is the whole array
        # unless some query has fewer than k records in its strides
        return out[:int(off[-1])], off


def cluster(queries, k_min: int = 2, k_max: int = 8, max_iter: int = 100, stream=None) -> dict:
    """Batch clustering (Section 4.4, Fig. 2) on the GPU: the chosen cluster
    count K, every target's label, the K centers, the k-medians rounds and the
    mean silhouette of every count tried (fps_cluster)."""
    torch = _require_gpu()
    c = load_library()
    qs = np.ascontiguousarray(np.asarray(queries, dtype=np.uint64).reshape(-1, 3))
    nq = qs.shape[0]
    nb = ctypes.c_size_t()
    _check(c.fps_cluster_workspace_bytes(nq, ctypes.byref(nb)))
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
    labels = np.zeros(nq, dtype=np.uint32)
    centers = np.zeros((max(k_max, 1), 3), dtype=np.uint64)
    info = ClusterInfo()
    _check(c.fps_cluster(_ptr(qs), nq, int(k_min), int(k_max), int(max_iter),
                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream),
                         _ptr(labels), _ptr(centers), ctypes.byref(info)))
    return _cluster_result(info, labels, centers, k_min, k_max)


class WideLibrary:
    """A library of wider fingerprints (W = 4, 8, 16 or 32 words: 256 to 2,048
    keys, every bit a key) resident in HBM (Section 5, concluding remark 3)."""

    def __init__(self, words: np.ndarray, strides=None, stream=None):
        torch = _require_gpu()
        c = load_library()
        w = np.ascontiguousarray(words, dtype=np.uint64)
        if w.ndim != 2:
            raise ValueError("words must be (n, W)")
        self.n, self.W = int(w.shape[0]), int(w.shape[1])
        nbytes = int(c.fps_wide_device_bytes(self.n, self.W))
        self._buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
        self._device = self._buf.device.index
        self._ws = None
        self._handle = ctypes.c_void_p()
        self.strides = [0, self.n] if strides is None else [int(x) for x in strides]
        st = None if strides is None else np.ascontiguousarray(strides, dtype=np.uint64)
        _check(c.fps_wide_load(_ptr(w), self.n, self.W, None if st is None else _ptr(st),
                               0 if st is None else len(st) - 1,
                               ctypes.c_void_p(self._buf.data_ptr()), nbytes, _stream(stream),
                               ctypes.byref(self._handle)))

    def close(self):
        if self._handle:
            load_library().fps_wide_free(self._handle)
            self._handle = ctypes.c_void_p()
        self._buf = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_path(self, path: int):
        _check(load_library().fps_wide_set_path(self._handle, int(path)))

    def set_tuning(self, candidate_scale: float = 1.0, sample_records: int = 0,
                   force_fallback: bool = False):
        _check(load_library().fps_wide_set_tuning(self._handle, float(candidate_scale),
                                                  int(sample_records), int(bool(force_fallback))))

    def set_timing(self, enable: bool):
        _check(load_library().fps_wide_set_timing(self._handle, int(bool(enable))))

    def last_stats(self) -> dict:
        st = SearchStats()
        _check(load_library().fps_wide_last_search_stats(self._handle, ctypes.byref(st)))
        return {"path": PATH_NAMES.get(st.path, st.path), "queries": st.queries,
                "fallbacks": st.fallbacks, "candidates": st.candidates, "scan_ms": st.scan_ms,
                "total_ms": st.total_ms, "scan_launches": st.scan_launches,
                "scan_ms_sum": st.scan_ms_sum, "total_ms_sum": st.total_ms_sum,
                "calls": st.calls}

    def _workspace(self, nbytes: int):
        import torch
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device="cuda")
        return self._ws

    def search_batch(self, queries, k, mask=None, stream=None):
        """Independent top-k per query: (hits, offsets), as Library.search_batch."""
        c = load_library()
        qs = np.ascontiguousarray(np.asarray(queries, dtype=np.uint64).reshape(-1, self.W))
        nq = qs.shape[0]
        kk = _u32(k, nq)
        mm = None if mask is None else _u32(mask, nq)
        nb = ctypes.c_size_t()
        _check(c.fps_wide_workspace_bytes(self._handle, nq, _ptr(kk),
                                          None if mm is None else _ptr(mm), ctypes.byref(nb)))
        ws = self._workspace(int(nb.value))
        cap = int(kk.astype(np.uint64).sum())
        out = np.empty(max(cap, 1), dtype=HIT_DTYPE)
        off = np.zeros(nq + 1, dtype=np.uint64)
        _check(c.fps_wide_search_batch(self._handle, _ptr(qs), nq, _ptr(kk),
                                       None if mm is None else _ptr(mm),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _ptr(out), cap,
                                       _ptr(off), _stream(stream, self._device)))
        return out[:int(off[-1])], off

    def search(self, query, k: int, mask: int = MASK_ALL, stream=None) -> np.ndarray:
        h, _ = self.search_batch(np.asarray(query).reshape(1, self.W), [k], [mask], stream)
        return h.copy()


def clock_ns() -> int:
    """Now on the steady clock of the server's time stamps (nanoseconds)."""
    return int(load_library().fps_clock_ns())


class Server:
    """Continuous-batching request loop over a Library (Sections 3.1, 4.4)."""

    def __init__(self, library: Library, pool_bytes: int, max_batch_queries: int = 512,
                 max_wait_us: int = 0, n_streams: int = 2, deadline_cap: bool = True,
                 reserve_streams: int = 0, tune_k=()):
        torch = _require_gpu()
        self._lib = library
        self._ws = torch.empty(int(pool_bytes), dtype=torch.uint8, device="cuda")
        tk = np.ascontiguousarray(np.asarray(tune_k, dtype=np.uint32).reshape(-1))
        cfg = ServerConfig(int(pool_bytes), int(max_batch_queries), int(max_wait_us),
                           int(n_streams), int(bool(deadline_cap)), int(reserve_streams),
                           ctypes.c_void_p(tk.ctypes.data) if len(tk) else None, len(tk))
        self._h = ctypes.c_void_p()
        _check(load_library().fps_server_create(library.handle, ctypes.byref(cfg),
                                                ctypes.c_void_p(self._ws.data_ptr()),
                                                int(pool_bytes), ctypes.byref(self._h)))

    def submit(self, queries, k: int, mask: int = MASK_ALL, deadline_us: int = 0,
               nonblocking: bool = False, arrival_ns: int = 0) -> int:
        """Queues a request; arrival_ns (clock_ns() time, 0 = now) is where its
        latency and deadline start."""
        qs = np.ascontiguousarray(np.asarray(queries, dtype=np.uint64).reshape(-1, 3))
        t = ctypes.c_uint64()
        _check(load_library().fps_server_submit(self._h, _ptr(qs), qs.shape[0], int(k),
                                                int(mask), int(deadline_us), int(arrival_ns),
                                                int(nonblocking), ctypes.byref(t)))
        return int(t.value)

    def wait(self, ticket: int):
        """Results of a request: (hits, offsets, stats), as Library.search_batch."""
        c = load_library()
        nq = ctypes.c_uint32()
        nh = ctypes.c_uint64()
        _check(c.fps_server_result_size(self._h, int(ticket), ctypes.byref(nq),
                                        ctypes.byref(nh)))
        out = np.empty(max(int(nh.value), 1), dtype=HIT_DTYPE)
        off = np.zeros(int(nq.value) + 1, dtype=np.uint64)
        st = RequestStats()
        _check(c.fps_server_wait(self._h, int(ticket), _ptr(out), int(nh.value), _ptr(off),
                                 len(off), ctypes.byref(st)))
        stats = {f: getattr(st, f) for f, _ in RequestStats._fields_}
        return out[:int(off[-1])], off, stats

    def stats(self, reset: bool = False) -> dict:
        st = ServerStats()
        _check(load_library().fps_server_stats_get(self._h, ctypes.byref(st), int(reset)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            load_library().fps_server_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
