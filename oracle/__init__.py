"""CPU oracle for the MESSI hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow definitions written from the paper (Peng, Fatourou, Palpanas,
"Fast Data Series Indexing for In-Memory Data"), in C (``messi_oracle.c``)
behind this ctypes wrapper.  Only the tests, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package; the GPU
library never calls it and shares no code with it.

All distances returned are squared, FP64, computed from the FP32
z-normalised values.  Parity unpinned: ``leaf_partition`` (the canonical
split order is this code's reading of Section 2.2; only its invariants,
Theorem 1, are fixed by the paper).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ED = 0
DTW = 1


class OracleLeaf(ctypes.Structure):
    _fields_ = [
        ("begin", ctypes.c_int64),
        ("end", ctypes.c_int64),
        ("sym", ctypes.c_uint8 * 16),
        ("bits", ctypes.c_uint8 * 16),
    ]


class SearchStats(ctypes.Structure):
    _fields_ = [
        ("leaves_total", ctypes.c_int64),
        ("leaves_enqueued", ctypes.c_int64),
        ("leaves_processed", ctypes.c_int64),
        ("series_lb", ctypes.c_int64),
        ("lb_keogh", ctypes.c_int64),
        ("real_dist", ctypes.c_int64),
        ("bsf_updates", ctypes.c_int64),
        ("approx_leaf", ctypes.c_int64),
        ("bsf_monotone", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (FP contraction off, OpenMP)."""
    import subprocess

    src = os.path.join(_HERE, "messi_oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
             "-fopenmp", "-shared", "-fPIC", "-o", tmp, src, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.oracle_znorm.argtypes = [P, i32, P]
        L.oracle_paa.argtypes = [P, i32, i32, P]
        L.oracle_breakpoints.argtypes = [i32, P]
        L.oracle_symbol.argtypes = [ctypes.c_float, P, i32]
        L.oracle_threads.restype = i32
        L.oracle_set_normalise.argtypes = [i32]
        L.oracle_symbol.restype = i32
        L.oracle_words.argtypes = [P, i64, i32, i32, i32, P]
        L.oracle_leaf_partition.argtypes = [P, i64, i32, i32, i32, P, P, i64]
        L.oracle_leaf_partition.restype = i64
        L.oracle_ed2.argtypes = [P, P, i32]
        L.oracle_ed2.restype = f64
        L.oracle_dtw2.argtypes = [P, P, i32, i32]
        L.oracle_dtw2.restype = f64
        L.oracle_envelope.argtypes = [P, i32, i32, P, P]
        L.oracle_lb_keogh2.argtypes = [P, P, P, i32]
        L.oracle_lb_keogh2.restype = f64
        L.oracle_mindist2_ed.argtypes = [P, P, P, P, i32, i32, i32]
        L.oracle_mindist2_ed.restype = f64
        L.oracle_mindist2_dtw.argtypes = [P, P, P, P, P, i32, i32, i32]
        L.oracle_mindist2_dtw.restype = f64
        L.oracle_knn_scan.argtypes = [P, i64, i64, i32, P, i32, i32, i32, i32, P, P]
        L.oracle_knn_scan_lbk.argtypes = [P, i64, i64, i32, P, i32, i32, i32, P, P]
        L.oracle_knn_scan_lbi.argtypes = [P, i64, i64, i32, P, i32, i32, i32, P, P]
        L.oracle_lb_improved2.argtypes = [P, P, P, P, i32, i32]
        L.oracle_lb_improved2.restype = f64
        L.oracle_knn_vote.argtypes = [P, i32, i32, P, i32, P]
        L.oracle_index_search.argtypes = [P, i64, i32, i32, i32, P, P, P, i64, P, i32, i32, i32,
                                          P, P, P]
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class raw_mode:
    """Context: series and queries are taken as given, not z-normalised."""

    def __enter__(self):
        lib().oracle_set_normalise(0)
        return self

    def __exit__(self, *exc):
        lib().oracle_set_normalise(1)
        return False


def windows(series, length, stride=1):
    """Rows of a subsequence index: the windows of `length` points of one
    long series, starting every `stride` points (Section 2.1)."""
    series = _f32(series)
    n = (len(series) - length) // stride + 1
    return np.stack([series[i * stride:i * stride + length] for i in range(n)])


def threads():
    """OpenMP threads the scans use."""
    return int(lib().oracle_threads())


def znorm(x):
    x = _f32(x)
    z = np.empty_like(x)
    for i in range(x.shape[0]) if x.ndim == 2 else [None]:
        if i is None:
            lib().oracle_znorm(_p(x), x.shape[-1], _p(z))
        else:
            lib().oracle_znorm(_p(x[i]), x.shape[-1], _p(z[i]))
    return z


def paa(z, w):
    z = _f32(z)
    out = np.empty(w, dtype=np.float32)
    lib().oracle_paa(_p(z), z.shape[-1], w, _p(out))
    return out


def breakpoints(card_bits=8):
    beta = np.empty((1 << card_bits) - 1, dtype=np.float32)
    lib().oracle_breakpoints(card_bits, _p(beta))
    return beta


def symbol(p, beta, card_bits=8):
    beta = _f32(beta)
    return int(lib().oracle_symbol(ctypes.c_float(p), _p(beta), card_bits))


def words(raw, w=16, card_bits=8):
    raw = _f32(raw)
    n, length = raw.shape
    out = np.empty((n, w), dtype=np.uint8)
    lib().oracle_words(_p(raw), n, length, w, card_bits, _p(out))
    return out


def leaf_partition(wds, leaf_size, card_bits=8):
    """Returns (perm int32[n], list of dict leaves with begin/end/sym/bits)."""
    wds = np.ascontiguousarray(wds, dtype=np.uint8)
    n, w = wds.shape
    perm = np.empty(max(n, 1), dtype=np.int32)
    cap = max(16, 4 * (n // max(1, leaf_size) + 1) + n // 4 + 64)
    while True:
        arr = (OracleLeaf * cap)()
        cnt = lib().oracle_leaf_partition(_p(wds), n, w, card_bits, leaf_size, _p(perm),
                                          ctypes.cast(arr, ctypes.c_void_p), cap)
        if cnt >= 0:
            break
        cap *= 4
    leaves = np.zeros(cnt, dtype=[("begin", np.int64), ("end", np.int64), ("sym", np.uint8, 16),
                                  ("bits", np.uint8, 16)])
    raw = np.ctypeslib.as_array(ctypes.cast(arr, ctypes.POINTER(ctypes.c_uint8)),
                                shape=(cap * ctypes.sizeof(OracleLeaf),))
    view = raw[: cnt * ctypes.sizeof(OracleLeaf)].view(leaves.dtype)
    leaves[:] = view
    return perm[:n].copy(), leaves


def ed2(q, x):
    q, x = _f32(q), _f32(x)
    return lib().oracle_ed2(_p(q), _p(x), q.shape[-1])


def dtw2(q, x, r):
    q, x = _f32(q), _f32(x)
    return lib().oracle_dtw2(_p(q), _p(x), q.shape[-1], int(r))


def envelope(q, r):
    q = _f32(q)
    U = np.empty_like(q)
    L = np.empty_like(q)
    lib().oracle_envelope(_p(q), q.shape[-1], int(r), _p(U), _p(L))
    return U, L


def lb_keogh2(U, L, x):
    U, L, x = _f32(U), _f32(L), _f32(x)
    return lib().oracle_lb_keogh2(_p(U), _p(L), _p(x), x.shape[-1])


def lb_improved2(q, U, L, x, r):
    q, U, L, x = _f32(q), _f32(U), _f32(L), _f32(x)
    return lib().oracle_lb_improved2(_p(q), _p(U), _p(L), _p(x), x.shape[-1], int(r))


def mindist2_ed(qpaa, sym, bits, beta, length, card_bits=8):
    qpaa, beta = _f32(qpaa), _f32(beta)
    sym = np.ascontiguousarray(sym, dtype=np.uint8)
    bits = np.ascontiguousarray(bits, dtype=np.uint8)
    return lib().oracle_mindist2_ed(_p(qpaa), _p(sym), _p(bits), _p(beta), qpaa.shape[0],
                                    length, card_bits)


def mindist2_dtw(upaa, lpaa, sym, bits, beta, length, card_bits=8):
    upaa, lpaa, beta = _f32(upaa), _f32(lpaa), _f32(beta)
    sym = np.ascontiguousarray(sym, dtype=np.uint8)
    bits = np.ascontiguousarray(bits, dtype=np.uint8)
    return lib().oracle_mindist2_dtw(_p(upaa), _p(lpaa), _p(sym), _p(bits), _p(beta),
                                     upaa.shape[0], length, card_bits)


class KnnState:
    """Running brute-force k-NN over a collection fed in chunks."""

    def __init__(self, raw_queries, k, distance=ED, r=0, lb_keogh=False, lb_improved=False):
        """lb_keogh / lb_improved: for DTW, skip pairs by LB_Keogh or by
        LB_Improved against the running k-th best (same lists, fewer DTW
        evaluations)."""
        self.lb_keogh = bool(lb_keogh) and int(distance) == DTW
        self.lb_improved = bool(lb_improved) and int(distance) == DTW
        self.q = _f32(raw_queries)
        self.nq, self.len = self.q.shape
        self.k, self.distance, self.r = int(k), int(distance), int(r)
        self.ids = np.full((self.nq, self.k), -1, dtype=np.int64)
        self.d2 = np.full((self.nq, self.k), np.inf, dtype=np.float64)

    def scan(self, raw_chunk, id0):
        raw_chunk = _f32(raw_chunk)
        if self.lb_improved:
            lib().oracle_knn_scan_lbi(_p(raw_chunk), int(id0), raw_chunk.shape[0], self.len,
                                      _p(self.q), self.nq, self.k, self.r, _p(self.ids),
                                      _p(self.d2))
            return self
        if self.lb_keogh:
            lib().oracle_knn_scan_lbk(_p(raw_chunk), int(id0), raw_chunk.shape[0], self.len,
                                      _p(self.q), self.nq, self.k, self.r, _p(self.ids),
                                      _p(self.d2))
            return self
        lib().oracle_knn_scan(_p(raw_chunk), int(id0), raw_chunk.shape[0], self.len, _p(self.q),
                              self.nq, self.k, self.distance, self.r, _p(self.ids), _p(self.d2))
        return self


def knn(raw, raw_queries, k, distance=ED, r=0):
    """Brute-force k-NN by definition: (ids int64[nq,k], d2 float64[nq,k])."""
    st = KnnState(raw_queries, k, distance, r).scan(raw, 0)
    return st.ids, st.d2


def knn_vote(ids, labels, n_classes):
    """Majority class of each k-NN list (ties: the class met first)."""
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    out = np.empty(ids.shape[0], dtype=np.int32)
    lib().oracle_knn_vote(_p(ids), ids.shape[0], ids.shape[1], _p(labels), int(n_classes), _p(out))
    return out


def index_search(raw, wds, perm, leaves, raw_query, k, distance=ED, r=0, card_bits=8):
    raw = _f32(raw)
    n, length = raw.shape
    w = wds.shape[1]
    wds = np.ascontiguousarray(wds, dtype=np.uint8)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    leaves = np.ascontiguousarray(leaves)
    q = _f32(raw_query)
    ids = np.empty(k, dtype=np.int64)
    d2 = np.empty(k, dtype=np.float64)
    st = SearchStats()
    lib().oracle_index_search(_p(raw), n, length, w, card_bits, _p(wds), _p(perm), _p(leaves),
                              len(leaves), _p(q), int(k), int(distance), int(r), _p(ids), _p(d2),
                              ctypes.cast(ctypes.pointer(st), ctypes.c_void_p))
    return ids, d2, st.as_dict()
