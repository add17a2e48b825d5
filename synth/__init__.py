"""Seeded synthetic workloads (random walks, noisy-copy queries).

This module holds no arithmetic of the indexing method: it only produces the
inputs that both the GPU library and the CPU oracle are fed.  The series
definition lives in ``randomwalk.h``; ``libsynth_host.so`` (gcc, OpenMP)
and ``libsynth_dev.so`` (hipcc, gfx950) are two builds of that one header
and produce the same bits.

Workload recipes (Sections 5.1 and 5.3 of the paper):
  * collection: random walks, x_0 ~ N(0,1), x_t = x_{t-1} + N(0,1), FP64
    cumulative sum rounded to FP32; series i of the collection is keyed by
    (seed 1, i);
  * random queries: the same generator with seed 2;
  * noisy queries: query j copies collection series synth_noisy_source_id(j)
    and adds N(0, (sigma * sd)^2) per point, sigma round robin over
    {0.01, 0.1, 1.0}, sd the series' own standard deviation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
HOST_LIB = os.path.join(_HERE, "libsynth_host.so")
DEV_LIB = os.path.join(_HERE, "libsynth_dev.so")

SEED_DATA = 1
SEED_QUERY = 2
SEED_NOISE = 3
SEED_MIX = 4
SEED_ARRIVAL = 5

_host = None
_dev = None


def build_host() -> str:
    tmp = HOST_LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off",
                           "-fno-fast-math", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                           os.path.join(_HERE, "synth_host.c")])
    os.replace(tmp, HOST_LIB)
    return HOST_LIB


def build_device(hipcc: str = "hipcc") -> str:
    tmp = DEV_LIB + ".tmp"
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O3", "-ffp-contract=off",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-fPIC", "-shared", "-o", tmp,
                           os.path.join(_HERE, "synth_device.hip")])
    os.replace(tmp, DEV_LIB)
    return DEV_LIB


def host():
    global _host
    if _host is None:
        if not os.path.exists(HOST_LIB):
            build_host()
        L = ctypes.CDLL(HOST_LIB)
        P, u64, i64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32
        L.synth_host_randomwalk.argtypes = [u64, u64, i64, i32, P]
        L.synth_host_noisy_queries.argtypes = [u64, u64, i32, u64, i64, P, P, P]
        L.synth_host_normals.argtypes = [u64, u64, i64, P]
        L.synth_host_uniforms.argtypes = [u64, u64, i64, P]
        L.synth_host_trend_labels.argtypes = [P, i64, i32, P]
        L.synth_host_log.argtypes = [ctypes.c_double]
        L.synth_host_log.restype = ctypes.c_double
        L.synth_host_sqrt.argtypes = [ctypes.c_double]
        L.synth_host_sqrt.restype = ctypes.c_double
        _host = L
    return _host


def device():
    global _dev
    if _dev is None:
        if not os.path.exists(DEV_LIB):
            raise RuntimeError("libsynth_dev.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(DEV_LIB)
        L.synth_dev_randomwalk.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                           ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
        L.synth_dev_randomwalk.restype = ctypes.c_int
        L.synth_dev_trend_labels.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_void_p]
        L.synth_dev_trend_labels.restype = ctypes.c_int
        _dev = L
    return _dev


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def randomwalk(count, length=256, seed=SEED_DATA, id0=0, out=None):
    """Series id0 .. id0+count-1 of the random-walk collection keyed by seed."""
    if out is None:
        out = np.empty((count, length), dtype=np.float32)
    assert out.dtype == np.float32 and out.flags.c_contiguous and out.shape == (count, length)
    host().synth_host_randomwalk(seed, id0, count, length, _p(out))
    return out


def random_queries(nq, length=256, seed=SEED_QUERY):
    return randomwalk(nq, length, seed=seed)


def noisy_queries(nq, n, length=256, data_seed=SEED_DATA, j0=0):
    """Noisy-copy queries j0 .. j0+nq-1 over a collection of n series.

    Returns (queries float32[nq, len], source ids int64[nq], sigmas float64[nq]).
    """
    out = np.empty((nq, length), dtype=np.float32)
    src = np.empty(nq, dtype=np.int64)
    sig = np.empty(nq, dtype=np.float64)
    host().synth_host_noisy_queries(data_seed, n, length, j0, nq, _p(out), _p(src), _p(sig))
    return out, src, sig


def trend_labels(raw):
    """Trend class (0..3) of each raw series: 2 [x_end > x_0] + [x_mid > x_0]."""
    raw = np.ascontiguousarray(raw, dtype=np.float32)
    out = np.empty(raw.shape[0], dtype=np.int32)
    host().synth_host_trend_labels(_p(raw), raw.shape[0], raw.shape[1], _p(out))
    return out


def trend_labels_device(tensor, out, stream=None):
    """Trend classes of a contiguous float32 CUDA tensor [n, len] into an
    int32 CUDA tensor [n]."""
    import torch

    assert tensor.is_cuda and tensor.is_contiguous() and tensor.dtype == torch.float32
    assert out.is_cuda and out.dtype == torch.int32 and out.numel() == tensor.shape[0]
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    rc = device().synth_dev_trend_labels(ctypes.c_void_p(tensor.data_ptr()), tensor.shape[0],
                                         tensor.shape[1], ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(s))
    if rc != 0:
        raise RuntimeError(f"synth_dev_trend_labels failed ({rc})")


def normals(count, seed=7, stream=0):
    out = np.empty(count, dtype=np.float64)
    host().synth_host_normals(seed, stream, count, _p(out))
    return out


def ar1_series(total, phi=0.995, seed=SEED_DATA, stream=11):
    """One long stationary series x_t = phi x_{t-1} + sqrt(1 - phi^2) e_t with
    e_t ~ N(0, 1) (x_0 = e_0): unit variance, locally like a random walk.
    The long input of subsequence search over values taken as they are."""
    from scipy.signal import lfilter

    e = normals(total, seed=seed, stream=stream)
    x = np.empty(total, dtype=np.float64)
    x[0] = e[0]
    if total > 1:  # the recursion as a one-pole filter started from x_0
        x[1:] = lfilter([np.sqrt(1.0 - phi * phi)], [1.0, -phi], e[1:], zi=[phi * e[0]])[0]
    return x.astype(np.float32)


def uniforms(count, seed=7, stream=0):
    out = np.empty(count, dtype=np.float64)
    host().synth_host_uniforms(seed, stream, count, _p(out))
    return out


def randomwalk_device(tensor, seed=SEED_DATA, id0=0, stream=None):
    """Fill a contiguous float32 CUDA tensor [count, len] on the GPU."""
    import torch

    assert tensor.is_cuda and tensor.dtype == torch.float32 and tensor.is_contiguous()
    count, length = tensor.shape
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    rc = device().synth_dev_randomwalk(seed, id0, count, length,
                                       ctypes.c_void_p(tensor.data_ptr()), ctypes.c_void_p(s))
    if rc != 0:
        raise RuntimeError(f"synth_dev_randomwalk failed with {rc}")
    return tensor
