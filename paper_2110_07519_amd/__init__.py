"""Python binding of libmessi (MESSI exact k-NN search on one MI355X).

Argument marshalling only: every step of the build and of a query runs in
the HIP kernels of libmessi.so behind the C ABI declared in
include/messi.h.  Torch is used for device memory and streams.  If the
library is not built, importing works but every call raises.

Names follow the C ABI: messi_build, messi_build_ex, messi_build_windows, messi_query, messi_query_stats,
messi_query_noalloc,
messi_query_batch, messi_autotune, messi_prepare_screen, messi_classify, messi_set_stream,
messi_free, messi_breakpoints, messi_get_words,
messi_get_perm, messi_get_leaves, messi_index_info, messi_build_times, messi_last_error.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmessi.so")

MESSI_OK = 0
MESSI_EINVAL = -1
MESSI_ENOMEM = -2
MESSI_EDEVICE = -3
MESSI_EBUSY = -4
MESSI_ED = 0
MESSI_DTW = 1
MESSI_SCREEN_BF16 = 1
MESSI_LB_IMPROVED = 2
MESSI_GRAPH = 4

EXPORTS = [
    "messi_build", "messi_query", "messi_query_stats", "messi_set_stream", "messi_index_info",
    "messi_build_times", "messi_get_words", "messi_get_perm", "messi_get_leaves",
    "messi_breakpoints", "messi_free", "messi_last_error", "messi_query_batch", "messi_prepare_screen",
    "messi_server_start", "messi_server_submit", "messi_server_poll", "messi_server_get_stats",
    "messi_server_stop", "messi_classify", "messi_build_ex", "messi_build_windows",
    "messi_query_noalloc", "messi_autotune",
]


class MessiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmessi error {code}: {msg}")
        self.code = code


class MessiLeaf(ctypes.Structure):
    _fields_ = [("begin", ctypes.c_int64), ("end", ctypes.c_int64),
                ("sym", ctypes.c_uint8 * 16), ("bits", ctypes.c_uint8 * 16)]


class MessiStats(ctypes.Structure):
    _fields_ = [("queries", ctypes.c_int64), ("leaves_total", ctypes.c_int64),
                ("leaves_kept", ctypes.c_int64), ("series_lb", ctypes.c_int64),
                ("lb_keogh", ctypes.c_int64), ("refined", ctypes.c_int64),
                ("rechecked_fp64", ctypes.c_int64), ("log_overflows", ctypes.c_int64),
                ("us_prep", ctypes.c_double), ("us_stage1", ctypes.c_double),
                ("us_process", ctypes.c_double), ("us_finalize", ctypes.c_double),
                ("screened", ctypes.c_int64), ("lb_improved", ctypes.c_int64),
                ("bsf_updates", ctypes.c_int64), ("dtw_cells", ctypes.c_int64),
                ("min_leaves", ctypes.c_int64), ("min_series", ctypes.c_int64),
                ("min_refined", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class MessiServerOptions(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("mem_budget_bytes", ctypes.c_int64), ("flags", ctypes.c_int32),
                ("kmax", ctypes.c_int32)]


class MessiServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("max_batch_seen", ctypes.c_int64),
                ("inflight_bytes", ctypes.c_int64), ("peak_inflight_bytes", ctypes.c_int64),
                ("mem_budget_bytes", ctypes.c_int64), ("request_bytes", ctypes.c_int64),
                ("batch_capacity", ctypes.c_int64), ("busy_us", ctypes.c_double),
                ("resident_bytes", ctypes.c_int64), ("log_growth_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib():
    """The loaded libmessi.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.messi_build.argtypes = [P, i64, i32, i32, i32, i32, ctypes.POINTER(P)]
        L.messi_build_ex.argtypes = [P, i64, i32, i32, i32, i32, P, ctypes.POINTER(P)]
        L.messi_build_windows.argtypes = [P, i64, i32, i32, i32, i32, i32, P, ctypes.POINTER(P)]
        L.messi_query.argtypes = [P, P, i32, i32, i32, i32, P, P]
        L.messi_query_stats.argtypes = [P, P, i32, i32, i32, i32, P, P, P]
        L.messi_query_noalloc.argtypes = [P, P, i32, i32, i32, i32, P, P]
        L.messi_query_batch.argtypes = [P, P, i32, P, P, P, i32, i32, P, P, P]
        L.messi_autotune.argtypes = [P, P, i32, P, P, P, i32, i32, P]
        L.messi_prepare_screen.argtypes = [P]
        L.messi_classify.argtypes = [P, P, i32, P, i32, i32, i32, i32, i32, P, P, P]
        L.messi_server_start.argtypes = [P, P, P]
        L.messi_server_submit.argtypes = [P, P, i32, i32, i32, P]
        L.messi_server_poll.argtypes = [P, i32, i32, P, P, P, P, P, P]
        L.messi_server_get_stats.argtypes = [P, P]
        L.messi_server_stop.argtypes = [P]
        L.messi_server_stop.restype = None
        L.messi_set_stream.argtypes = [P, P]
        L.messi_index_info.argtypes = [P, P, P, P, P, P, P]
        L.messi_build_times.argtypes = [P, P, P]
        L.messi_get_words.argtypes = [P, P]
        L.messi_get_perm.argtypes = [P, P]
        L.messi_get_leaves.argtypes = [P, P, i64, P]
        L.messi_breakpoints.argtypes = [i32, P]
        L.messi_free.argtypes = [P]
        L.messi_free.restype = None
        L.messi_last_error.restype = ctypes.c_char_p
        for name in ["messi_build", "messi_build_ex", "messi_build_windows", "messi_query", "messi_query_stats",
                     "messi_query_noalloc", "messi_query_batch", "messi_autotune",
                     "messi_prepare_screen", "messi_classify", "messi_server_start",
                     "messi_server_submit",
                     "messi_server_poll", "messi_server_get_stats", "messi_set_stream",
                     "messi_index_info", "messi_build_times", "messi_get_words", "messi_get_perm",
                     "messi_get_leaves", "messi_breakpoints"]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != MESSI_OK:
        raise MessiError(rc, lib().messi_last_error().decode())


def _dev_ptr(t):
    import torch

    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def messi_breakpoints(card_bits: int = 8) -> np.ndarray:
    beta = np.empty((1 << card_bits) - 1, dtype=np.float32)
    _check(lib().messi_breakpoints(card_bits, beta.ctypes.data_as(ctypes.c_void_p)))
    return beta


def messi_build(series, segments: int = 16, cardinality: int = 256, leaf_size: int = 2000):
    """Build an index over a float32 CUDA tensor [n, len]; returns an Index."""
    import torch

    assert series.dtype == torch.float32 and series.dim() == 2
    n, length = series.shape
    h = ctypes.c_void_p()
    _check(lib().messi_build(_dev_ptr(series), n, length, segments, cardinality, leaf_size,
                             ctypes.byref(h)))
    return Index(h, n, length, segments)


class MessiOptions(ctypes.Structure):
    _fields_ = [("inplace", ctypes.c_int32), ("bf16_screen", ctypes.c_int32),
                ("raw", ctypes.c_int32), ("mem_budget_bytes", ctypes.c_int64),
                ("autotune_cache", ctypes.c_char_p)]


class MessiTune(ctypes.Structure):
    _fields_ = [("screen", ctypes.c_int32), ("screen_min", ctypes.c_int32),
                ("screen_nt", ctypes.c_int32), ("screen_occ", ctypes.c_int32),
                ("ed_scale", ctypes.c_int32), ("dtw_scale", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("screen_waves", ctypes.c_int32),
                ("ms", ctypes.c_double), ("ms_default", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def _options(inplace=0, bf16_screen=False, raw=False, mem_budget_bytes=0, autotune_cache=None):
    path = None if autotune_cache is None else os.fsencode(autotune_cache)
    return MessiOptions(int(inplace), int(bf16_screen), int(raw), int(mem_budget_bytes), path)


def messi_build_ex(series, segments: int = 16, cardinality: int = 256, leaf_size: int = 2000,
                   inplace: bool = False, bf16_screen: bool = False, raw: bool = False,
                   mem_budget_bytes: int = 0, autotune_cache=None):
    """messi_build with options.  inplace: `series` (float32 CUDA [n, len]) is
    z-normalised in place and becomes the store; keep it alive and unmodified
    while the index lives (the returned Index holds a reference).  raw: the
    series (and later the queries) are used as given, not z-normalised.
    mem_budget_bytes: device bytes the index may hold (0: no limit).
    autotune_cache: path of the JSON file of tuned batch knobs."""
    import torch

    assert series.dtype == torch.float32 and series.dim() == 2
    n, length = series.shape
    h = ctypes.c_void_p()
    o = _options(int(inplace), bf16_screen, raw, mem_budget_bytes, autotune_cache)
    _check(lib().messi_build_ex(_dev_ptr(series), n, length, segments, cardinality, leaf_size,
                                ctypes.cast(ctypes.pointer(o), ctypes.c_void_p), ctypes.byref(h)))
    idx = Index(h, n, length, segments)
    if inplace:
        idx.store = series
    return idx


def messi_build_owned(ptr: int, n: int, length: int, segments: int = 16, cardinality: int = 256,
                      leaf_size: int = 2000, bf16_screen: bool = False, raw: bool = False,
                      mem_budget_bytes: int = 0, autotune_cache=None):
    """In-place build that hands the device buffer at `ptr` (the start of a
    hipMalloc allocation of n * length float32) over to the index, which
    frees it in messi_free (messi_options.inplace = 2)."""
    h = ctypes.c_void_p()
    o = _options(2, bf16_screen, raw, mem_budget_bytes, autotune_cache)
    _check(lib().messi_build_ex(ctypes.c_void_p(ptr), n, length, segments, cardinality, leaf_size,
                                ctypes.cast(ctypes.pointer(o), ctypes.c_void_p), ctypes.byref(h)))
    return Index(h, n, length, segments)


def messi_build_windows(series, length: int, stride: int = 1, segments: int = 16,
                        cardinality: int = 256, leaf_size: int = 2000, raw: bool = True,
                        bf16_screen: bool = False):
    """Index every window of `length` points (window starts `stride` apart)
    of one long float32 CUDA series [total]; id i of an answer is the window
    starting at i * stride.  raw (the default here): windows as given."""
    import torch

    assert series.dtype == torch.float32 and series.dim() == 1 and series.is_contiguous()
    total = series.shape[0]
    h = ctypes.c_void_p()
    o = _options(1, bf16_screen, raw)
    _check(lib().messi_build_windows(_dev_ptr(series), total, length, stride, segments, cardinality,
                                     leaf_size, ctypes.cast(ctypes.pointer(o), ctypes.c_void_p),
                                     ctypes.byref(h)))
    return Index(h, (total - length) // stride + 1, length, segments)


def messi_query(index, queries, k: int = 1, distance: int = MESSI_ED, window: int = 0,
                out_ids=None, out_dists=None, stats: bool = False):
    """Exact k-NN of float32 CUDA queries [nq, len]: (ids int64 [nq,k], dists float32 [nq,k])."""
    import torch

    assert queries.dtype == torch.float32 and queries.dim() == 2
    nq = queries.shape[0]
    dev = queries.device
    if out_ids is None:
        out_ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
    if out_dists is None:
        out_dists = torch.empty((nq, k), dtype=torch.float32, device=dev)
    if not stats:
        _check(lib().messi_query(index.handle, _dev_ptr(queries), nq, k, distance, window,
                                 _dev_ptr(out_ids), _dev_ptr(out_dists)))
        return out_ids, out_dists
    st = MessiStats()
    _check(lib().messi_query_stats(index.handle, _dev_ptr(queries), nq, k, distance, window,
                                   _dev_ptr(out_ids), _dev_ptr(out_dists),
                                   ctypes.cast(ctypes.pointer(st), ctypes.c_void_p)))
    return out_ids, out_dists, st.as_dict()


def messi_query_noalloc(index, queries, k: int = 1, distance: int = MESSI_ED, window: int = 0,
                        out_ids=None, out_dists=None):
    """messi_query whose query state lives in the library's fixed scratch
    array (no device allocation by the library during the call)."""
    import torch

    assert queries.dtype == torch.float32 and queries.dim() == 2
    nq = queries.shape[0]
    dev = queries.device
    if out_ids is None:
        out_ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
    if out_dists is None:
        out_dists = torch.empty((nq, k), dtype=torch.float32, device=dev)
    _check(lib().messi_query_noalloc(index.handle, _dev_ptr(queries), nq, k, distance, window,
                                     _dev_ptr(out_ids), _dev_ptr(out_dists)))
    return out_ids, out_dists


def messi_query_batch(index, queries, k, distance, window, kmax=None, flags=0, out_ids=None,
                      out_dists=None, stats: bool = False):
    """Batch with per-query k / distance / window (sequences of nq ints):
    (ids int64 [nq,kmax], dists float32 [nq,kmax][, stats])."""
    import torch

    assert queries.dtype == torch.float32 and queries.dim() == 2
    nq = queries.shape[0]
    kk = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int32), (nq,)))
    dd = np.ascontiguousarray(np.broadcast_to(np.asarray(distance, dtype=np.int32), (nq,)))
    ww = np.ascontiguousarray(np.broadcast_to(np.asarray(window, dtype=np.int32), (nq,)))
    if kmax is None:
        kmax = int(kk.max()) if nq else 1
    dev = queries.device
    if out_ids is None:
        out_ids = torch.empty((nq, kmax), dtype=torch.int64, device=dev)
    if out_dists is None:
        out_dists = torch.empty((nq, kmax), dtype=torch.float32, device=dev)
    st = MessiStats() if stats else None
    sp = ctypes.cast(ctypes.pointer(st), ctypes.c_void_p) if stats else None
    _check(lib().messi_query_batch(index.handle, _dev_ptr(queries), nq,
                                   kk.ctypes.data_as(ctypes.c_void_p),
                                   dd.ctypes.data_as(ctypes.c_void_p),
                                   ww.ctypes.data_as(ctypes.c_void_p), int(kmax), int(flags),
                                   _dev_ptr(out_ids), _dev_ptr(out_dists), sp))
    if stats:
        return out_ids, out_dists, st.as_dict()
    return out_ids, out_dists


def messi_autotune(index, queries, k, distance, window, kmax=None, flags=0) -> dict:
    """Tune messi_query_batch's knobs on this batch (arguments as for
    messi_query_batch); returns the chosen knobs and the timings."""
    import torch

    assert queries.dtype == torch.float32 and queries.dim() == 2
    nq = queries.shape[0]
    kk = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int32), (nq,)))
    dd = np.ascontiguousarray(np.broadcast_to(np.asarray(distance, dtype=np.int32), (nq,)))
    ww = np.ascontiguousarray(np.broadcast_to(np.asarray(window, dtype=np.int32), (nq,)))
    if kmax is None:
        kmax = int(kk.max()) if nq else 1
    t = MessiTune()
    _check(lib().messi_autotune(index.handle, _dev_ptr(queries), nq, kk.ctypes.data_as(ctypes.c_void_p),
                                dd.ctypes.data_as(ctypes.c_void_p), ww.ctypes.data_as(ctypes.c_void_p),
                                int(kmax), int(flags), ctypes.byref(t)))
    return t.as_dict()


def messi_classify(index, labels, n_classes, queries, k=1, distance=MESSI_ED, window=0, flags=0):
    """k-NN classification of float32 CUDA queries [nq, len] with int32 CUDA
    labels [n]: (classes int32 [nq], ids int64 [nq, k], dists float32 [nq, k])."""
    import torch

    assert queries.dtype == torch.float32 and queries.dim() == 2 and labels.dtype == torch.int32
    nq = queries.shape[0]
    dev = queries.device
    cls = torch.empty(nq, dtype=torch.int32, device=dev)
    ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
    d = torch.empty((nq, k), dtype=torch.float32, device=dev)
    _check(lib().messi_classify(index.handle, _dev_ptr(labels), int(n_classes), _dev_ptr(queries), nq,
                                int(k), int(distance), int(window), int(flags), _dev_ptr(cls),
                                _dev_ptr(ids), _dev_ptr(d)))
    return cls, ids, d


def messi_prepare_screen(index) -> None:
    _check(lib().messi_prepare_screen(index.handle))


def messi_set_stream(index, stream) -> None:
    _check(lib().messi_set_stream(index.handle, ctypes.c_void_p(stream)))


def messi_free(index) -> None:
    if index.handle:
        lib().messi_free(index.handle)
        index.handle = None


def messi_index_info(index) -> dict:
    n, ln, w, cb, nl, db = (ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(),
                            ctypes.c_int64(), ctypes.c_int64())
    _check(lib().messi_index_info(index.handle, ctypes.byref(n), ctypes.byref(ln), ctypes.byref(w),
                                  ctypes.byref(cb), ctypes.byref(nl), ctypes.byref(db)))
    return {"n": n.value, "len": ln.value, "segments": w.value, "card_bits": cb.value,
            "n_leaves": nl.value, "device_bytes": db.value}


def messi_build_times(index) -> dict:
    """Host wall time of the build call, and its part in device allocation (ms)."""
    t, a = ctypes.c_double(), ctypes.c_double()
    _check(lib().messi_build_times(index.handle, ctypes.byref(t), ctypes.byref(a)))
    return {"build_ms": t.value, "alloc_ms": a.value}


def messi_get_words(index) -> np.ndarray:
    out = np.empty((index.n, index.segments), dtype=np.uint8)
    _check(lib().messi_get_words(index.handle, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def messi_get_perm(index) -> np.ndarray:
    out = np.empty(index.n, dtype=np.int32)
    _check(lib().messi_get_perm(index.handle, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def messi_get_leaves(index) -> np.ndarray:
    cnt = ctypes.c_int64()
    info = messi_index_info(index)
    cap = info["n_leaves"]
    arr = (MessiLeaf * max(cap, 1))()
    _check(lib().messi_get_leaves(index.handle, ctypes.cast(arr, ctypes.c_void_p), cap,
                                  ctypes.byref(cnt)))
    dt = np.dtype([("begin", np.int64), ("end", np.int64), ("sym", np.uint8, 16),
                   ("bits", np.uint8, 16)])
    raw = np.frombuffer(arr, dtype=np.uint8, count=cnt.value * ctypes.sizeof(MessiLeaf))
    return raw.view(dt).copy()


class Server:
    """Serving loop over a built index (messi_server_*): submit() queues a
    host query, poll() returns finished requests as
    (request id, status, ids[k], dists[k], latency in microseconds)."""

    def __init__(self, index, workers=2, max_batch=1024, mem_budget_bytes=0, flags=0, kmax=64):
        o = MessiServerOptions(workers, max_batch, mem_budget_bytes, flags, kmax)
        h = ctypes.c_void_p()
        _check(lib().messi_server_start(index.handle, ctypes.byref(o), ctypes.byref(h)))
        self.handle, self.index, self.kmax, self.len = h, index, kmax, index.len

    def submit(self, query, k=1, distance=MESSI_ED, window=0) -> int:
        q = np.ascontiguousarray(query, dtype=np.float32).reshape(-1)
        assert q.shape[0] == self.len
        rid = ctypes.c_uint64()
        _check(lib().messi_server_submit(self.handle, q.ctypes.data_as(ctypes.c_void_p), int(k),
                                         int(distance), int(window), ctypes.byref(rid)))
        return rid.value

    def poll(self, max_results=256, timeout_ms=0):
        rid = np.empty(max_results, dtype=np.uint64)
        stt = np.empty(max_results, dtype=np.int32)
        ids = np.empty((max_results, self.kmax), dtype=np.int64)
        dd = np.empty((max_results, self.kmax), dtype=np.float32)
        lat = np.empty(max_results, dtype=np.float64)
        cnt = ctypes.c_int32()
        P = ctypes.c_void_p
        _check(lib().messi_server_poll(self.handle, max_results, int(timeout_ms),
                                       rid.ctypes.data_as(P), stt.ctypes.data_as(P),
                                       ids.ctypes.data_as(P), dd.ctypes.data_as(P),
                                       lat.ctypes.data_as(P), ctypes.byref(cnt)))
        return [(int(rid[i]), int(stt[i]), ids[i].copy(), dd[i].copy(), float(lat[i]))
                for i in range(cnt.value)]

    def stats(self):
        st = MessiServerStats()
        _check(lib().messi_server_get_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def stop(self):
        if self.handle:
            lib().messi_server_stop(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


class Index:
    """Owning handle of a built index."""

    def __init__(self, handle, n, length, segments):
        self.handle = handle
        self.n, self.len, self.segments = n, length, segments

    def query(self, queries, k=1, distance=MESSI_ED, window=0, stats=False):
        return messi_query(self, queries, k, distance, window, stats=stats)

    def info(self):
        return messi_index_info(self)

    def free(self):
        messi_free(self)

    def __del__(self):
        try:
            messi_free(self)
        except Exception:
            pass
