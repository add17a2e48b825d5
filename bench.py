#!/usr/bin/env python3
"""Benchmark of the MESSI hot path on one MI355X.

Workload (the paper's default collection, Section 5.1): 100,000,000 random
walks of length 256 in FP32 (102.4 GB, generated in HBM by the seeded device
generator), iSAX index with 16 segments, 8-bit symbols, leaves of 2000;
random-walk queries from a separate seed answered one at a time (exact 1-NN,
Euclidean distance).  A step is one query through the whole hot path
(preparation, approximate search, leaf bounds, leaf processing with series
bounds and refinement, FP64 near-tie recheck).  Also reported: index build
time (after a small build that loads the kernels; build_alloc_s is its part
in hipMalloc, which grows when earlier processes left the device's memory
to be cleared before reuse), per-phase device times, the roofline of the dominant kernel, the CPU
oracle timed on a sample, exact 1-NN DTW (radius 25 = 10% of 256) over the
first 10,000,000 series and over the whole collection with noisy dataset
copies as queries (noise 0.01, 0.1, 1.0 times the series' standard
deviation, round robin), and batches of 1,024 noisy copies through the
plain path, the BF16 screen and graph replay at 100M x 256 and, built in
place, at 200M x 128.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 MFMA, published
# Plain (unpacked) FP32 VALU issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz,
# in tera lane-instructions per second (the DTW kernels use no packed ops)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU instructions of one DTW band cell on gfx950: the difference, the
# minimum of the three neighbours (one v_min3) and the fused square-and-add
# (the masked bands, which the default radius does not use, add a median)
DTW_OPS_PER_CELL = 3

# HBM bytes per launch of the ED process kernel, from two rocprofv3 --pmc
# runs of this script (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 KiB; factors from
# a 1 GiB device copy and fill), keyed by the timed query set (steps,
# warmup): valid only for those queries and for the query kernel sources
# they were taken on.
MEASURED_TRAFFIC = {"sources_sha256": "e35e65eeea00f26705ee9bd3d8b5d7be6635f85c08a7a1f696c6f2aa0c1199c1",
                    "by_queries": {"100,5": 338851973, "20,5": 258084741}}
QUERY_SOURCES = ["paper_2110_07519_amd/csrc/query.hip", "paper_2110_07519_amd/csrc/query.h",
                 "paper_2110_07519_amd/csrc/common.h"]
PHASES = ["prep", "stage1", "process", "finalize"]


def query_sources_digest():
    import hashlib

    h = hashlib.sha256()
    for rel in QUERY_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def process_bytes(st, length, queries):
    """Algorithmic bytes per launch of the process kernel (one query per
    launch): the work the search needs once its final k-th best is known --
    the 16 B word of every series in a leaf whose bound is within it, and
    the 4 len B row of every such series whose own bound is within it.
    Also the bytes of the work the kernel did with its running k-th best."""
    q = max(queries, 1)
    row = 4 * length
    minimal = (16.0 * st["min_series"] + row * st["min_refined"]) / q
    running = (16.0 * st["series_lb"] + row * (st["refined"] + st["lb_keogh"])) / q
    return minimal, running


def run_queries(pm, idx, qt, k, distance, window, budget_s=None):
    """One messi_query per query (the production call through the C ABI, no
    statistics, into output buffers allocated once, as a serving loop
    would); returns wall seconds and per-query latencies."""
    import torch

    import ctypes

    lat = []
    out_ids = torch.empty((1, k), dtype=torch.int64, device=qt.device)
    out_dists = torch.empty((1, k), dtype=torch.float32, device=qt.device)
    # the C entry point with its arguments converted once, as a serving loop
    # holds them
    call = pm.lib().messi_query
    handle = idx.handle
    oi, od = ctypes.c_void_p(out_ids.data_ptr()), ctypes.c_void_p(out_dists.data_ptr())
    rows = [ctypes.c_void_p(qt[j:j + 1].data_ptr()) for j in range(qt.shape[0])]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for j in range(qt.shape[0]):
        t0 = time.perf_counter()
        rc = call(handle, rows[j], 1, k, distance, window, oi, od)
        if rc != pm.MESSI_OK:
            raise pm.MessiError(rc, pm.lib().messi_last_error().decode())
        lat.append(time.perf_counter() - t0)
        if budget_s is not None and time.perf_counter() - t_start > budget_s:
            break
    torch.cuda.synchronize()
    return time.perf_counter() - t_start, np.array(lat)


def query_stats(pm, idx, qt, k, distance, window):
    """The same queries again through messi_query_stats (untimed): work
    counters and per-phase device times (HIP events on the index's stream)."""
    tot = {}
    for j in range(qt.shape[0]):
        _, _, st = pm.messi_query(idx, qt[j:j + 1], k, distance, window, stats=True)
        for key, v in st.items():
            tot[key] = tot.get(key, 0) + v
    return tot


def run_c4(pm, idx, n, length, nq, reps):
    """The batched configuration on one index: one call per batch of nq
    noisy-copy queries (noise 0.01/0.1/1.0 round robin), ED, k alternating
    1 and 10.  The autotuner first picks the batch knobs for this shape
    (or finds them in its cache); then, best of reps: the plain FP32 path
    with the default knobs, the BF16 screen with the tuned knobs, and the
    same replayed from a HIP graph.  Answers of all three must be
    identical."""
    import torch
    import synth

    bq, _, _ = synth.noisy_queries(nq, n, length, j0=100_000)
    ks = [1 if i % 2 == 0 else 10 for i in range(nq)]
    bt = torch.from_numpy(bq).cuda()
    out = {"workload": f"{nq} noisy dataset copies per call over {n} x {length}, ED, k alternating 1 and 10",
           "n": n, "len": length, "batch": nq}
    t0 = time.perf_counter()
    pm.messi_prepare_screen(idx)
    torch.cuda.synchronize()
    out["screen_prepare_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    tune = pm.messi_autotune(idx, bt, ks, 0, 0, kmax=10, flags=pm.MESSI_SCREEN_BF16)
    out["autotune"] = dict(tune, seconds=time.perf_counter() - t0)
    log(f"C4 {n} x {length}: autotune {out['autotune']}")
    oi = torch.empty((nq, 10), dtype=torch.int64, device="cuda")
    od = torch.empty((nq, 10), dtype=torch.float32, device="cuda")
    answers = {}
    runs = (("plain", 0), ("screen", pm.MESSI_SCREEN_BF16), ("screen_graph", pm.MESSI_SCREEN_BF16 | pm.MESSI_GRAPH))
    for name, flags in runs:
        pm.messi_query_batch(idx, bt, ks, 0, 0, kmax=10, flags=flags, out_ids=oi, out_dists=od)  # warm / capture
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pm.messi_query_batch(idx, bt, ks, 0, 0, kmax=10, flags=flags, out_ids=oi, out_dists=od)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        answers[name] = (oi.cpu().numpy(), od.cpu().numpy())
        out[name] = {"queries_per_s": nq / best, "ms_per_batch": best * 1e3}
        if name != "screen_graph":  # phase times and counters from one more (untimed) call
            _, _, st = pm.messi_query_batch(idx, bt, ks, 0, 0, kmax=10, flags=flags, stats=True)
            out[name].update({"phases_us": {p: st[f"us_{p}"] for p in PHASES},
                              "refined_per_query": st["refined"] / nq,
                              "series_lb_per_query": st["series_lb"] / nq,
                              "screened_pairs_per_query": st["screened"] / nq})
        log(f"C4 {n} x {length} {name}: {nq / best:.0f} q/s ({best * 1e3:.1f} ms per {nq})")
    sc = out["screen"]
    if sc["screened_pairs_per_query"] > 0:
        flops = sc["screened_pairs_per_query"] * nq * 2.0 * length
        us = sc["phases_us"]["process"]
        sc["mfma_roofline"] = {"bound": "mfma", "achieved": flops / (us * 1e-6) / 1e12,
                               "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": flops / (us * 1e-6) / 1e12 / BF16_PEAK_TFLOPS,
                               "flops_per_launch": flops,
                               "note": "algorithmic q.x flops (2 len per screened pair) over the screen "
                                       "phase (leaf lists + screen kernel)"}
    ref = answers["plain"]
    out["identical_answers"] = bool(all(np.array_equal(ref[0], a[0]) and np.array_equal(ref[1], a[1])
                                        for a in answers.values()))
    out["screen_speedup"] = out["screen"]["queries_per_s"] / out["plain"]["queries_per_s"]
    out["graph_speedup"] = out["screen_graph"]["queries_per_s"] / out["screen"]["queries_per_s"]
    return out


def run_c4_200m(pm, n, length, nq, reps, cache):
    """The batched configuration at 200,000,000 x 128 (the SALD shape),
    generated in HBM and indexed in place."""
    import torch
    import synth

    log(f"C4: generating {n} x {length} random walks in HBM")
    data = torch.empty((n, length), dtype=torch.float32, device="cuda")
    synth.randomwalk_device(data, seed=synth.SEED_DATA)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx = pm.messi_build_ex(data, 16, 256, 2000, inplace=True, autotune_cache=cache)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    out = run_c4(pm, idx, n, length, nq, reps)
    out["build_s"] = build_s
    idx.free()
    del data
    torch.cuda.empty_cache()
    return out


SWEEP_SHAPES = [  # (series, length, in place): about 100 GB at every length, then sizes at 256
    (200_000_000, 128, 0), (100_000_000, 256, 0), (50_000_000, 512, 0), (25_000_000, 1024, 0),
    (12_500_000, 2048, 0), (50_000_000, 256, 0), (100_000_000, 256, 1), (150_000_000, 256, 1),
    (200_000_000, 256, 1),
]


def sweep_one(pm, args):
    """One sweep shape: build time and exact 1-NN ED queries/s, one query at
    a time, over random walks (the same generator and seeds as the default
    run)."""
    import torch
    import synth

    parts = [int(x) for x in args.sweep_one.split(",")]
    n, length, inplace = parts[0], parts[1], (parts[2] if len(parts) > 2 else 0)
    data = torch.empty((n, length), dtype=torch.float32, device="cuda")
    synth.randomwalk_device(data, seed=synth.SEED_DATA)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx = pm.messi_build_ex(data, 16, 256, args.leaf, inplace=bool(inplace))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    del data  # the in-place index keeps its own reference to the store
    torch.cuda.empty_cache()
    qt = torch.from_numpy(synth.random_queries(args.warmup + 50, length)).cuda()
    run_queries(pm, idx, qt[:args.warmup], 1, pm.MESSI_ED, 0)
    wall, lat = run_queries(pm, idx, qt[args.warmup:], 1, pm.MESSI_ED, 0)
    st = query_stats(pm, idx, qt[args.warmup:], 1, pm.MESSI_ED, 0)
    nqs = len(lat)
    idx.free()
    return {"n": n, "len": length, "inplace": bool(inplace), "gb": n * length * 4 / 1e9,
            "build_s": build_s,
            "queries_per_s": nqs / wall, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "series_lb_per_query": st["series_lb"] / nqs, "refined_per_query": st["refined"] / nqs}


def run_sweep(args):
    """Size and length sweep (the paper's Section 5.3 sweeps), one child
    process per shape."""
    import subprocess

    rows = []
    for n, length, inplace in SWEEP_SHAPES:
        cmd = [sys.executable, os.path.abspath(__file__), "--sweep-one", f"{n},{length},{inplace}",
               "--leaf", str(args.leaf), "--warmup", str(args.warmup)]
        res = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=600)
        if res.returncode != 0:
            raise RuntimeError(f"sweep shape {n} x {length} failed ({res.returncode})")
        row = json.loads(res.stdout.strip().splitlines()[-1])
        rows.append(row)
        log(f"sweep {n} x {length}{' in place' if inplace else ''}: build {row['build_s']:.3f} s, "
            f"{row['queries_per_s']:.0f} q/s, "
            f"p50 {row['p50_ms']:.3f} ms")
    ref = [r for r in rows if r["n"] == 100_000_000 and r["len"] == 256 and not r["inplace"]][0]
    return {"metric": "exact 1-NN queries/s (ED, one query at a time), size and length sweep",
            "value": ref["queries_per_s"], "unit": "queries/s", "n_gpus": 1, "steps": 50,
            "warmup": args.warmup, "ms_per_step": 1e3 / ref["queries_per_s"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic", "config": {"workload": "random-walk collections, 16 segments, 8-bit "
                                                        "iSAX, leaf 2000; 50 random-walk queries per shape"},
            "sweep": rows}


def run_classification(pm, idx, labels, n, length, nq):
    """k-NN classification (Section 5.4) of nq noisy dataset copies, ED,
    BF16 screen, k in {1, 10, 50}: queries/s per k, and agreement of the
    vote with the trend class of each query's source series."""
    import torch
    import synth

    qs, src, _ = synth.noisy_queries(nq, n, length, j0=400_000)
    qt = torch.from_numpy(qs).cuda()
    truth = labels[torch.from_numpy(src).cuda()].cpu().numpy()
    out = {"workload": f"{nq} noisy dataset copies per call, ED, BF16 screen; classes = trend "
                       "shape of the generated series (4 classes)", "k": []}
    for k in (1, 10, 50):
        pm.messi_classify(idx, labels, 4, qt[:32], k, flags=pm.MESSI_SCREEN_BF16)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cls, _, _ = pm.messi_classify(idx, labels, 4, qt, k, flags=pm.MESSI_SCREEN_BF16)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        acc = float((cls.cpu().numpy() == truth).mean())
        out["k"].append({"k": k, "queries_per_s": nq / dt, "ms_per_call": dt * 1e3,
                         "agreement_with_source_class": acc})
        log(f"classification k={k}: {nq / dt:.0f} q/s, agreement {acc:.3f}")
    return out


def serving_mix(count, n, length, j0):
    """Request mix: ED / DTW 50/50, DTW window 5/10/20% of the length, k 1 or
    10, noisy dataset copies (noise 0.01/0.1/1.0 round robin); seed 4."""
    import synth

    qs, _, _ = synth.noisy_queries(count, n, length, j0=j0)
    rng = np.random.default_rng(synth.SEED_MIX + j0)
    dist = rng.integers(0, 2, count)
    wins = [int(length * f) for f in (0.05, 0.10, 0.20)]
    win = np.where(dist == 1, rng.choice(wins, count), 0)
    ks = rng.choice([1, 10], count)
    return qs, [int(x) for x in ks], [int(x) for x in dist], [int(x) for x in win]


def run_serving(pm, idx, n, length, seconds, cap_requests):
    """Poisson arrivals of the request mix at 0.25, 0.5, 1 and 2 times the
    capacity of the unbatched plain path (one messi_query per request),
    served by the continuous-batching server; latency is arrival to result."""
    import threading

    import torch
    import synth

    qs, ks, dist, win = serving_mix(cap_requests, n, length, 200_000)
    qt = torch.from_numpy(qs).cuda()
    pm.messi_query(idx, qt[:1], 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(cap_requests):
        pm.messi_query(idx, qt[i:i + 1], ks[i], dist[i], win[i])
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / cap_requests
    capacity = 1.0 / plain_s
    log(f"serving: plain path {capacity:.1f} requests/s on the mix (one at a time)")
    out = {"workload": "Poisson arrivals; ED/DTW 50/50, DTW window 5/10/20%, k 1/10, noise "
                       "0.01/0.1/1.0; 2 workers, continuous batching, BF16 screen for ED",
           "plain_unbatched_requests_per_s": capacity, "capacity_sample": cap_requests,
           "rates": []}
    last = None
    srv = pm.Server(idx, workers=2, max_batch=1024, mem_budget_bytes=16 << 30,
                    flags=pm.MESSI_SCREEN_BF16, kmax=10)
    j0 = 300_000
    for f in (0.25, 0.5, 1.0, 2.0):
        lam = f * capacity
        cnt = max(20, int(lam * seconds))
        rq, rk, rd, rw = serving_mix(cnt, n, length, j0)
        last = (rq, rk, rd, rw)
        j0 += cnt
        gaps = np.random.default_rng(synth.SEED_ARRIVAL).exponential(1.0 / lam, cnt)
        lat = []

        def producer():
            t_next = time.perf_counter()
            for i in range(cnt):
                t_next += gaps[i]
                dt = t_next - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                srv.submit(rq[i], rk[i], rd[i], rw[i])

        t_start = time.perf_counter()
        th = threading.Thread(target=producer)
        th.start()
        t_limit = t_start + seconds * 4 + 60
        while len(lat) < cnt and time.perf_counter() < t_limit:
            for r in srv.poll(256, timeout_ms=20):
                assert r[1] == 0, "serving request failed"
                lat.append(r[4])
        th.join()
        wall = time.perf_counter() - t_start
        lat = np.array(lat) / 1e3
        row = {"rate_factor": f, "offered_requests_per_s": lam, "requests": cnt,
               "completed": int(len(lat)), "achieved_requests_per_s": len(lat) / wall,
               "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99))}
        out["rates"].append(row)
        log(f"serving at {f} x capacity ({lam:.1f}/s): {row['achieved_requests_per_s']:.1f}/s, "
            f"p50 {row['p50_ms']:.1f} ms, p99 {row['p99_ms']:.1f} ms")
    st = srv.stats()
    srv.stop()
    out["batches"] = st["batches"]
    out["max_batch_seen"] = st["max_batch_seen"]
    # the plain path on exactly the requests of the heaviest stream, one at a time
    rq, rk, rd, rw = last
    rt = torch.from_numpy(rq).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(len(rk)):
        pm.messi_query(idx, rt[i:i + 1], rk[i], rd[i], rw[i])
    torch.cuda.synchronize()
    same = len(rk) / (time.perf_counter() - t0)
    out["plain_unbatched_same_requests_per_s"] = same
    out["served_vs_plain_at_2x"] = out["rates"][-1]["achieved_requests_per_s"] / same
    log(f"serving: plain path on the 2x stream's {len(rk)} requests: {same:.1f}/s")
    return out


def dtw_filters(pm, idx, qt, window):
    """The same DTW queries one per messi_query_batch call, with LB_Keogh
    alone and with LB_Improved after it (MESSI_LB_IMPROVED): queries/s and
    the work each filter leaves."""
    import torch

    nq = qt.shape[0]
    out = {}
    for name, flags in (("lb_keogh", 0), ("lb_improved", pm.MESSI_LB_IMPROVED)):
        pm.messi_query_batch(idx, qt[:1], [1], [1], [window], flags=flags)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(nq):
            pm.messi_query_batch(idx, qt[j:j + 1], [1], [1], [window], flags=flags)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tot = {}
        for j in range(nq):
            _, _, st = pm.messi_query_batch(idx, qt[j:j + 1], [1], [1], [window], flags=flags,
                                            stats=True)
            for key, v in st.items():
                tot[key] = tot.get(key, 0) + v
        out[name] = {"queries_per_s": nq / dt, "lb_keogh_per_query": tot["lb_keogh"] / nq,
                     "lb_improved_per_query": tot["lb_improved"] / nq,
                     "dtw_per_query": tot["refined"] / nq,
                     "process_us": tot["us_process"] / nq}
        log(f"DTW {name}: {nq / dt:.1f} q/s, DTW {tot['refined'] / nq:.0f}/query, "
            f"LB_Improved {tot['lb_improved'] / nq:.0f}/query")
    return out


def run_subsequence(pm, total, length, nq):
    """Subsequence search (Section 2.1): every window of `length` points of
    one long series, indexed by messi_build_windows, raw values and
    z-normalised windows; exact 1-NN ED of noisy window copies, one query
    at a time."""
    import torch
    import synth

    s = synth.ar1_series(total)
    st = torch.from_numpy(s).cuda()
    rng = np.random.default_rng(synth.SEED_MIX)
    starts = rng.integers(0, total - length, nq + 3)
    qs = np.stack([s[a:a + length] for a in starts])
    qs += (0.1 * rng.standard_normal(qs.shape)).astype(np.float32)
    qt = torch.from_numpy(qs).cuda()
    out = {"workload": f"AR(1) series (phi 0.995, unit variance) of {total} points, every window "
                       f"of {length} (stride 1); {nq} window copies + N(0, 0.1^2) noise, "
                       "exact 1-NN ED one at a time", "modes": []}
    for as_given in (True, False):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        idx = pm.messi_build_windows(st, length, 1, leaf_size=2000, raw=as_given)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        run_queries(pm, idx, qt[:3], 1, pm.MESSI_ED, 0)
        wall, lat = run_queries(pm, idx, qt[3:], 1, pm.MESSI_ED, 0, budget_s=60)
        k = len(lat)
        stt = query_stats(pm, idx, qt[3:3 + k], 1, pm.MESSI_ED, 0)
        row = {"raw": as_given, "windows": idx.n, "build_s": build_s, "queries_per_s": k / wall,
               "p50_ms": float(np.percentile(lat, 50) * 1e3),
               "refined_per_query": stt["refined"] / k, "leaves_kept_per_query": stt["leaves_kept"] / k}
        out["modes"].append(row)
        log(f"subsequence raw={as_given}: {idx.n} windows, build {build_s:.3f} s, "
            f"{k / wall:.0f} q/s, refined {row['refined_per_query']:.0f}/query")
        idx.free()
    return out


def cpu_baseline(n, length, queries, sample):
    """The oracle's brute-force scan on the host cores over the first
    `sample` series (regenerated on the host in chunks; only the scans are
    timed), scaled to the whole collection."""
    import oracle
    import synth

    log(f"cpu baseline: oracle scan of {queries.shape[0]} queries over {sample} x {length}")
    st = oracle.KnnState(queries, 1)
    dt = 0.0
    chunk = 2_000_000
    for c in range(0, sample, chunk):
        raw = synth.randomwalk(min(chunk, sample - c), length, seed=synth.SEED_DATA, id0=c)
        t0 = time.perf_counter()
        st.scan(raw, c)
        dt += time.perf_counter() - t0
    cores = oracle.threads()
    qps = queries.shape[0] / dt * (sample / n)
    return {"value": qps, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "sample": f"brute-force exact 1-NN ED (FP64) of {queries.shape[0]} queries over the first "
                      f"{sample} of the {n} series: {dt:.1f} s of scanning, scaled by {sample}/{n}"}


def cpu_baseline_dtw(n, length, window, nq, sample):
    """The oracle's LB_Keogh-filtered DTW scan (exact; LB_Keogh against the
    running k-th best prunes pairs before the banded DTW) on the host cores,
    nq of the DTW run's noisy queries (noise 0.01/0.1/1.0 round robin) over
    the first `sample` of its n series (regenerated on the host; only the
    scans are timed), scaled to the n series.  A scan over fewer series
    prunes less, so the scaled rate understates the host."""
    import oracle
    import synth

    dq, _, _ = synth.noisy_queries(nq + 3, n, length)
    queries = dq[3:]
    log(f"cpu baseline: oracle LB_Keogh-filtered DTW (r={window}) of {nq} queries over "
        f"{sample} x {length}")
    st = oracle.KnnState(queries, 1, distance=oracle.DTW, r=window, lb_keogh=True)
    dt = 0.0
    chunk = 500_000
    for c in range(0, sample, chunk):
        raw = synth.randomwalk(min(chunk, sample - c), length, seed=synth.SEED_DATA, id0=c)
        t0 = time.perf_counter()
        st.scan(raw, c)
        dt += time.perf_counter() - t0
    return {"value": nq / dt * (sample / n), "unit": "queries/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"LB_Keogh-filtered exact 1-NN DTW (FP64, r={window}) of {nq} noisy queries "
                      f"over the first {sample} of the {n} series: {dt:.1f} s of scanning, "
                      f"scaled by {sample}/{n}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--len", type=int, default=256)
    ap.add_argument("--leaf", type=int, default=2000)
    ap.add_argument("--dtw-n", type=int, default=10_000_000)
    ap.add_argument("--dtw-queries", type=int, default=100)
    ap.add_argument("--window", type=int, default=25)
    ap.add_argument("--dtw-full-queries", type=int, default=30,
                    help="DTW queries on the full collection (noisy copies, one at a time)")
    ap.add_argument("--batch", type=int, default=1024,
                    help="queries of the batched run (noisy copies, k alternating 1 and 10)")
    ap.add_argument("--batch-reps", type=int, default=2)
    ap.add_argument("--c4-200m", type=int, default=200_000_000,
                    help="series of the 128-point batched configuration (0: skip it)")
    ap.add_argument("--autotune-cache", type=str, default=os.path.join("/tmp", "messi_autotune.json"),
                    help="JSON file of tuned batch knobs (read at build, written by the autotuner)")
    ap.add_argument("--classify", type=int, default=1024,
                    help="queries per k-NN classification call (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=6.0,
                    help="length of each Poisson arrival stream of the serving run (0: skip)")
    ap.add_argument("--serve-capacity-requests", type=int, default=40)
    ap.add_argument("--subseq-points", type=int, default=20_000_000,
                    help="length of the long series of the subsequence run (0 = skip)")
    ap.add_argument("--subseq-queries", type=int, default=100)
    ap.add_argument("--cpu-sample", type=int, default=16_000_000)
    ap.add_argument("--cpu-queries", type=int, default=100)
    ap.add_argument("--cpu-dtw-sample", type=int, default=1_000_000)
    ap.add_argument("--cpu-dtw-queries", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="size and length sweep instead of the default run (one JSON line)")
    ap.add_argument("--sweep-one", type=str, default="",
                    help="internal: one sweep shape 'n,len[,inplace]' in this process")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the index is built and "
              "queried on a single MI355X", file=sys.stderr)
        sys.exit(2)

    if args.sweep:  # each shape in a child process, so every build starts from a clean allocator
        print(json.dumps(run_sweep(args)), flush=True)
        return

    import torch

    import paper_2110_07519_amd as pm
    import synth

    n, length = args.n, args.len
    torch.cuda.init()
    if args.sweep_one:
        print(json.dumps(sweep_one(pm, args)), flush=True)
        return
    if args.copy_probe_mib > 0:
        a = torch.empty(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        a.fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del a, b
    log(f"generating {n} x {length} random walks in HBM")
    data = torch.empty((n, length), dtype=torch.float32, device="cuda")
    synth.randomwalk_device(data, seed=synth.SEED_DATA)
    torch.cuda.synchronize()
    dtw_n = min(args.dtw_n, n)
    didx = None
    if args.dtw_queries > 0:
        log(f"building the DTW index over the first {dtw_n} series")
        didx = pm.messi_build(data[:dtw_n], 16, 256, args.leaf)
        torch.cuda.synchronize()
    labels = None
    if args.classify > 0:
        labels = torch.empty(n, dtype=torch.int32, device="cuda")
        synth.trend_labels_device(data, labels)
    # a small build first loads the library's kernels (done once per process)
    pm.messi_build(data[:100000], 16, 256, args.leaf).free()
    log("building the index")
    t0 = time.perf_counter()
    idx = pm.messi_build_ex(data, 16, 256, args.leaf, autotune_cache=args.autotune_cache)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = idx.info()
    bt = pm.messi_build_times(idx)
    log(f"build {build_s:.3f} s ({bt['alloc_ms']:.1f} ms of it in device allocation), "
        f"{info['n_leaves']} leaves")
    del data
    torch.cuda.empty_cache()

    nq = args.warmup + args.steps
    qs = synth.random_queries(nq, length)
    qt = torch.from_numpy(qs).cuda()
    log(f"warmup {args.warmup} queries")
    run_queries(pm, idx, qt[:args.warmup], 1, pm.MESSI_ED, 0)
    log(f"timing {args.steps} ED queries one at a time")
    wall, lat = run_queries(pm, idx, qt[args.warmup:], 1, pm.MESSI_ED, 0)
    k_done = len(lat)
    st = query_stats(pm, idx, qt[args.warmup:args.warmup + k_done], 1, pm.MESSI_ED, 0)
    value = k_done / wall
    phases_us = {p: st[f"us_{p}"] / k_done for p in PHASES}
    dom_bytes, run_bytes = process_bytes(st, length, k_done)
    achieved = dom_bytes / (phases_us["process"] * 1e-6) / 1e9
    log(f"ED: {value:.1f} q/s, p50 {np.percentile(lat, 50) * 1e3:.3f} ms, phases {phases_us}")

    dtw = None
    if didx is not None:
        dq, _, dsig = synth.noisy_queries(args.dtw_queries + 3, dtw_n, length)
        dt = torch.from_numpy(dq).cuda()
        run_queries(pm, didx, dt[:3], 1, pm.MESSI_DTW, args.window)
        log(f"timing {args.dtw_queries} DTW queries (r={args.window}) over {dtw_n} series")
        dwall, dlat = run_queries(pm, didx, dt[3:], 1, pm.MESSI_DTW, args.window, budget_s=90)
        dk = len(dlat)
        dst = query_stats(pm, didx, dt[3:3 + dk], 1, pm.MESSI_DTW, args.window)
        dph = {p: dst[f"us_{p}"] / dk for p in PHASES}
        ops = dst["dtw_cells"] / dk * DTW_OPS_PER_CELL
        dach = ops / (dph["process"] * 1e-6) / 1e12
        dtw_roof = {"kernel": f"k_process (register band, radius {args.window})", "bound": "alu",
                    "achieved": dach, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                    "frac": dach / VALU_PEAK_TOPS, "traffic": None,
                    "ops_per_launch": ops, "cells_per_launch": dst["dtw_cells"] / dk,
                    "note": f"{DTW_OPS_PER_CELL} VALU instructions per band cell computed (v_sub, v_min3, "
                            "v_fmac; cells "
                            "counted in the kernel: rows done before each pair ended, within the "
                            "band and the matrix) over the process phase; peak = plain FP32 VALU "
                            "issue of 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz"}
        dtw = {"metric": "exact 1-NN DTW queries/s (one query at a time)", "value": dk / dwall,
               "unit": "queries/s", "queries": dk, "window": args.window,
               "workload": f"first {dtw_n} of the random walks, noisy dataset copies "
                           "(noise 0.01/0.1/1.0 x series sd, round robin)",
               "p50_ms": float(np.percentile(dlat, 50) * 1e3),
               "p99_ms": float(np.percentile(dlat, 99) * 1e3), "phases_us": dph,
               "refined_per_query": dst["refined"] / dk, "lb_keogh_per_query": dst["lb_keogh"] / dk,
               "series_lb_per_query": dst["series_lb"] / dk,
               "bsf_updates_per_query": dst["bsf_updates"] / dk,
               "roofline": dtw_roof}
        log(f"DTW: {dtw['value']:.2f} q/s, p50 {dtw['p50_ms']:.2f} ms, p99 {dtw['p99_ms']:.2f} ms")
        dtw["filters"] = dtw_filters(pm, didx, dt[3:3 + dk], args.window)
        didx.free()

    dtw_full = None
    if args.dtw_full_queries > 0:
        fq, _, _ = synth.noisy_queries(args.dtw_full_queries + 2, n, length, j0=200_000)
        ft = torch.from_numpy(fq).cuda()
        run_queries(pm, idx, ft[:2], 1, pm.MESSI_DTW, args.window)
        log(f"timing {args.dtw_full_queries} DTW queries (r={args.window}) over all {n} series")
        fwall, flat = run_queries(pm, idx, ft[2:], 1, pm.MESSI_DTW, args.window, budget_s=60)
        fk = len(flat)
        fst = query_stats(pm, idx, ft[2:2 + fk], 1, pm.MESSI_DTW, args.window)
        dtw_full = {"metric": "exact 1-NN DTW queries/s (one query at a time)", "value": fk / fwall,
                    "unit": "queries/s", "queries": fk, "window": args.window,
                    "workload": f"all {n} random walks, noisy dataset copies (noise 0.01/0.1/1.0 x "
                                "series sd, round robin)",
                    "p50_ms": float(np.percentile(flat, 50) * 1e3),
                    "p99_ms": float(np.percentile(flat, 99) * 1e3),
                    "phases_us": {p: fst[f"us_{p}"] / fk for p in PHASES},
                    "refined_per_query": fst["refined"] / fk, "lb_keogh_per_query": fst["lb_keogh"] / fk}
        log(f"DTW at {n}: {dtw_full['value']:.2f} q/s, p50 {dtw_full['p50_ms']:.2f} ms, "
            f"p99 {dtw_full['p99_ms']:.2f} ms")

    batched = None
    if args.batch > 0:
        batched = {f"{n // 1_000_000}Mx{length}": run_c4(pm, idx, n, length, args.batch, args.batch_reps)}

    classification = None
    if labels is not None:
        classification = run_classification(pm, idx, labels, n, length, args.classify)
        del labels

    serving = None
    if args.serve_seconds > 0:
        serving = run_serving(pm, idx, n, length, args.serve_seconds, args.serve_capacity_requests)

    idx.free()
    torch.cuda.empty_cache()
    if args.batch > 0 and args.c4_200m > 0:
        batched[f"{args.c4_200m // 1_000_000}Mx128"] = run_c4_200m(pm, args.c4_200m, 128, args.batch,
                                                                  args.batch_reps, args.autotune_cache)

    subsequence = None
    if args.subseq_points > 0:
        subsequence = run_subsequence(pm, args.subseq_points, length, args.subseq_queries)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(n, length, qs[args.warmup:args.warmup + args.cpu_queries],
                           min(args.cpu_sample, n))
        log(f"cpu baseline {cpu['value']:.4f} q/s")
        if args.dtw_queries > 0 and args.cpu_dtw_queries > 0:
            cpu["dtw"] = cpu_baseline_dtw(dtw_n, length, args.window, args.cpu_dtw_queries,
                                          min(args.cpu_dtw_sample, dtw_n))
            log(f"cpu baseline DTW {cpu['dtw']['value']:.4f} q/s")

    traffic = None
    if MEASURED_TRAFFIC["sources_sha256"] == query_sources_digest():
        traffic = MEASURED_TRAFFIC["by_queries"].get(f"{args.steps},{args.warmup}")
    out = {
        "metric": "exact 1-NN queries/s (ED, one query at a time)",
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": k_done,
        "warmup": args.warmup,
        "ms_per_step": wall / k_done * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"random-walk collection {n} x {length} FP32 in HBM, 16 segments, "
                               f"8-bit iSAX, leaf {args.leaf}; random-walk queries, exact 1-NN ED, "
                               f"one at a time", "n": n, "len": length, "leaf_size": args.leaf,
                   "k": 1},
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "build_s": build_s,
        "build_alloc_s": bt["alloc_ms"] / 1e3,
        "n_leaves": info["n_leaves"],
        "phases_us": phases_us,
        "work_per_query": {"leaves_kept": st["leaves_kept"] / k_done,
                           "series_lb": st["series_lb"] / k_done,
                           "refined": st["refined"] / k_done,
                           "rechecked_fp64": st["rechecked_fp64"] / k_done,
                           "bsf_updates": st["bsf_updates"] / k_done,
                           "min_leaves": st["min_leaves"] / k_done,
                           "min_series": st["min_series"] / k_done,
                           "min_refined": st["min_refined"] / k_done},
        "roofline": {"kernel": "k_process_ed", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": dom_bytes,
                     "bytes_per_launch_running_kth": run_bytes,
                     "note": "bytes_per_launch: 16 B per series in a leaf within the final k-th "
                             "best + 4 len B per series whose own bound is within it (the work "
                             "the search needs once the answer is known); the kernel did "
                             "bytes_per_launch_running_kth with its running k-th best"},
        "dtw": dtw,
        "dtw_full": dtw_full,
        "batched": batched,
        "classification": classification,
        "serving": serving,
        "subsequence": subsequence,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
