"""GPU parity at the benchmark sizes, in the benchmark's launch configuration.

* Exact 1-NN ED over 100,000,000 random walks of length 256 (16 segments,
  8-bit symbols, leaves of 2000): 100 random-walk queries answered one at
  a time plus two noisy copies, a 10-NN call over the same queries, the
  10-NN classifier's vote, and a screened batch of 37 (rows equal to single
  calls).  On the same index, a batch of 1,024 noisy copies (noise 0.01 /
  0.1 / 1.0, k alternating 1 and 10) through the BF16 screen with tuned
  knobs and graph replay: every row equals the plain batch's and a single
  call's, and 32 rows spread over the batch are checked by the oracle.
  Two noisy copies (noise 0.01 and 0.1) answered under DTW (r = 25) over
  the whole collection.  One host scan of the whole collection
  (regenerated in chunks by the seeded generator) answers every oracle
  query (DTW through the LB_Keogh-filtered scan).
* Exact 1-NN DTW (radius 25) over 10,000,000 random walks of length 256:
  nine noisy dataset copies (noise 0.01, 0.1 and 1.0), each checked
  against the oracle's LB_Keogh-filtered scan (equal to the plain scan,
  pinned on the CPU).
* The same 1,024-query batch at 200,000,000 x 128 (index built in place):
  rows equal to the plain batch and to single calls, 32 of them checked by
  the oracle's scan.

The device collection comes from the seeded device generator, which is
bitwise equal to the host generator (test_device_generator_matches_host).
"""
import contextlib
import sys
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")

CHUNK = 2_000_000


_capsys = None


def _say(msg):
    """Progress on the terminal even while pytest captures output (a long
    silent test would look hung)."""
    if _capsys is not None:
        with _capsys.disabled():
            print(f"[scale] {msg}", file=sys.stderr, flush=True)
    else:
        print(f"[scale] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(autouse=True)
def _progress(capsys):
    global _capsys
    _capsys = capsys
    yield
    _capsys = None


@pytest.fixture(scope="module")
def pm():
    import paper_2110_07519_amd as pm

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pm.lib()
    return pm


def _device_index(pm, n, length, leaf, labels=None):
    data = torch.empty((n, length), dtype=torch.float32, device="cuda")
    synth.randomwalk_device(data, seed=synth.SEED_DATA)
    if labels is not None:  # trend classes of the collection, for the classifier
        synth.trend_labels_device(data, labels)
    idx = pm.messi_build(data, 16, 256, leaf)
    torch.cuda.synchronize()
    del data
    torch.cuda.empty_cache()
    return idx


def _host_scan(states, n, length):
    t0 = last = time.perf_counter()
    for c in range(0, n, CHUNK):
        raw = synth.randomwalk(min(CHUNK, n - c), length, seed=synth.SEED_DATA, id0=c)
        for st in states:
            st.scan(raw, c)
        if time.perf_counter() - last > 20:
            last = time.perf_counter()
            _say(f"oracle scanned {c + len(raw)} / {n} series ({last - t0:.0f} s)")


def _check(ids, d, oids, od2):
    assert np.array_equal(ids, oids), (ids, oids)
    od = np.sqrt(od2)
    assert np.all(np.abs(d - od) <= 1e-4 * np.maximum(od, 1e-3)), (d, od)


def _host_rows(a):
    return a.cpu().numpy()


def _c4_batch(pm, idx, n, length, nq=1024):
    """The 1,024-query batch of noisy copies (k alternating 1 and 10) with
    the screen, tuned and replayed from a graph, against the plain batch
    and single calls.  Returns (queries, ks, ids, dists, rows for the
    oracle)."""
    qs, _, _ = synth.noisy_queries(nq, n, length, j0=100_000)
    ks = [1 if i % 2 == 0 else 10 for i in range(nq)]
    qt = torch.from_numpy(qs).cuda()
    tune = pm.messi_autotune(idx, qt, ks, 0, 0, kmax=10, flags=pm.MESSI_SCREEN_BF16)
    _say(f"C4 {n} x {length}: tuned {tune}")
    plain = [_host_rows(t) for t in pm.messi_query_batch(idx, qt, ks, 0, 0, kmax=10)]
    out_i = torch.empty((nq, 10), dtype=torch.int64, device="cuda")
    out_d = torch.empty((nq, 10), dtype=torch.float32, device="cuda")
    for _ in range(2):  # capture, then replay
        pm.messi_query_batch(idx, qt, ks, 0, 0, kmax=10, flags=pm.MESSI_SCREEN_BF16 | pm.MESSI_GRAPH,
                             out_ids=out_i, out_dists=out_d)
        torch.cuda.synchronize()
        assert np.array_equal(_host_rows(out_i), plain[0]) and np.array_equal(_host_rows(out_d), plain[1])
    for i in range(nq):
        sid, sd = pm.messi_query(idx, qt[i:i + 1], ks[i])
        assert np.array_equal(plain[0][i, :ks[i]], _host_rows(sid)[0]), i
        assert np.array_equal(plain[1][i, :ks[i]], _host_rows(sd)[0]), i
    assert np.all(plain[0][0::2, 1:] == -1)
    rows = np.arange(0, nq, nq // 32)
    return qs, ks, plain[0], plain[1], rows


def test_ed_100m_one_query_at_a_time_and_batch(pm):
    n, length = 100_000_000, 256
    _say(f"ED: building the index over {n} x {length}")
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    idx = _device_index(pm, n, length, 2000, labels)
    qn, _, _ = synth.noisy_queries(3, n, length)  # noise 0.01, 0.1, 1.0
    qs = np.concatenate([synth.random_queries(100, length), qn[[0, 2]]])
    qt = torch.from_numpy(qs).cuda()
    one = [pm.messi_query(idx, qt[j:j + 1], 1) for j in range(len(qs))]
    ids1 = np.concatenate([o[0].cpu().numpy() for o in one])
    d1 = np.concatenate([o[1].cpu().numpy() for o in one])
    ids10, d10 = (t.cpu().numpy() for t in pm.messi_query(idx, qt, 10))
    cls, cids, _ = pm.messi_classify(idx, labels, 4, qt, 10)  # k-NN classifier, k = 10
    cls, cids = cls.cpu().numpy(), cids.cpu().numpy()
    del labels
    pm.messi_prepare_screen(idx)
    # a screened batch of 37 (5 of these and 32 noisy copies, k 10 / 3):
    # rows equal to one call per query
    qb = np.concatenate([qs[:5], synth.noisy_queries(32, n, length, j0=1000)[0]])
    qbt = torch.from_numpy(qb).cuda()
    kb = [10] * 5 + [3] * 32
    bids, bd, bst = pm.messi_query_batch(idx, qbt, kb, [0] * 37, [0] * 37, flags=pm.MESSI_SCREEN_BF16,
                                         stats=True)
    bids, bd = bids.cpu().numpy(), bd.cpu().numpy()
    assert bst["screened"] > 0
    for j in range(37):
        sid, sd = pm.messi_query(idx, qbt[j:j + 1], kb[j])
        assert np.array_equal(bids[j, :kb[j]], sid.cpu().numpy()[0]) and np.array_equal(bd[j, :kb[j]], sd.cpu().numpy()[0])
    cq, cks, cids4, cd4, rows = _c4_batch(pm, idx, n, length)
    # DTW (r = 25) over the whole collection: copies with noise 0.01 and
    # 0.1 of series in the first chunk the host scans (so that the oracle's
    # LB_Keogh-filtered scan has its k-th best early; the answer does not
    # depend on the scan's order)
    dq = np.concatenate([synth.noisy_queries(1, n, length, j0=j)[0] for j in (200961, 202441)])
    dqt = torch.from_numpy(dq).cuda()
    dres = [pm.messi_query(idx, dqt[j:j + 1], 1, pm.MESSI_DTW, 25) for j in range(2)]
    dids = np.concatenate([o[0].cpu().numpy() for o in dres])
    dd = np.concatenate([o[1].cpu().numpy() for o in dres])
    idx.free()
    _say(f"ED: GPU answers ready; oracle scan of the whole collection ({len(qs)} + {len(rows)} queries)")
    st = oracle.KnnState(qs, 10)
    st4 = oracle.KnnState(cq[rows], 10)
    std = oracle.KnnState(dq, 1, oracle.DTW, 25, lb_keogh=True)
    _host_scan([st, st4, std], n, length)
    _check(dids, dd, std.ids, std.d2)
    _check(ids1, d1, st.ids[:, :1], st.d2[:, :1])
    _check(ids10, d10, st.ids, st.d2)
    for t, i in enumerate(rows):
        _check(cids4[i:i + 1, :cks[i]], cd4[i:i + 1, :cks[i]], st4.ids[t:t + 1, :cks[i]], st4.d2[t:t + 1, :cks[i]])
    # the classifier's vote against the oracle's over the oracle's neighbours
    # (labels computed on the host for just those series; -1 elsewhere)
    assert np.array_equal(cids, st.ids)
    host_labels = np.full(n, -1, dtype=np.int32)
    for i in np.unique(st.ids):
        host_labels[i] = synth.trend_labels(synth.randomwalk(1, length, seed=synth.SEED_DATA, id0=int(i)))[0]
    assert np.array_equal(cls, oracle.knn_vote(st.ids, host_labels, 4))


def test_dtw_10m_noisy_queries(pm):
    n, length, r = 10_000_000, 256, 25
    _say(f"DTW: building the index over {n} x {length}")
    idx = _device_index(pm, n, length, 2000)
    qs, src, sig = synth.noisy_queries(9, n, length)  # noise 0.01, 0.1, 1.0 round robin
    assert sorted(set(np.round(sig, 2))) == [0.01, 0.1, 1.0]
    qt = torch.from_numpy(qs).cuda()
    one = [pm.messi_query(idx, qt[j:j + 1], 1, pm.MESSI_DTW, r) for j in range(len(qs))]
    ids = np.concatenate([o[0].cpu().numpy() for o in one])
    d = np.concatenate([o[1].cpu().numpy() for o in one])
    idx.free()
    _say("DTW: GPU answers ready; oracle scan (LB_Keogh-filtered DTW)")
    st = oracle.KnnState(qs, 1, oracle.DTW, r, lb_keogh=True)
    _host_scan([st], n, length)
    _check(ids, d, st.ids, st.d2)


def test_c4_batch_200m_by_128(pm):
    n, length = 200_000_000, 128
    _say(f"C4: generating and building in place over {n} x {length}")
    data = torch.empty((n, length), dtype=torch.float32, device="cuda")
    synth.randomwalk_device(data, seed=synth.SEED_DATA)
    idx = pm.messi_build_ex(data, 16, 256, 2000, inplace=True, bf16_screen=True)
    torch.cuda.synchronize()
    cq, cks, cids, cd, rows = _c4_batch(pm, idx, n, length)
    idx.free()
    del data
    torch.cuda.empty_cache()
    _say(f"C4: GPU answers ready; oracle scan of {n} x {length} ({len(rows)} queries)")
    st = oracle.KnnState(cq[rows], 10)
    _host_scan([st], n, length)
    for t, i in enumerate(rows):
        _check(cids[i:i + 1, :cks[i]], cd[i:i + 1, :cks[i]], st.ids[t:t + 1, :cks[i]], st.d2[t:t + 1, :cks[i]])


def test_subsequence_windows_20m_points(pm):
    """Subsequence search at the benchmark's size: every window of 256 points
    (stride 1) of a 20,000,000-point AR(1) series, raw and z-normalised,
    window copies plus N(0, 0.1^2) noise as queries, exact 5-NN ED against
    the oracle's scan over the same windows (cut from the host series in
    chunks)."""
    total, length = 20_000_000, 256
    s = synth.ar1_series(total)
    st_dev = torch.from_numpy(s).cuda()
    rng = np.random.default_rng(synth.SEED_MIX)
    starts = rng.integers(0, total - length, 6)
    qs = np.stack([s[a:a + length] for a in starts])
    qs[3:] += (0.1 * rng.standard_normal((3, length))).astype(np.float32)
    qt = torch.from_numpy(qs).cuda()
    nwin = total - length + 1
    view = np.lib.stride_tricks.sliding_window_view(s, length)
    for as_given in (True, False):
        _say(f"windows: building the {'raw' if as_given else 'z-normalised'} index over {nwin} windows")
        idx = pm.messi_build_windows(st_dev, length, 1, leaf_size=2000, raw=as_given)
        assert idx.n == nwin
        one = [pm.messi_query(idx, qt[j:j + 1], 5) for j in range(len(qs))]
        ids = np.concatenate([o[0].cpu().numpy() for o in one])
        d = np.concatenate([o[1].cpu().numpy() for o in one])
        idx.free()
        st = oracle.KnnState(qs, 5)
        t0 = time.perf_counter()
        with (oracle.raw_mode() if as_given else contextlib.nullcontext()):
            for c in range(0, nwin, CHUNK):
                st.scan(np.ascontiguousarray(view[c:c + CHUNK]), c)
        _say(f"windows: oracle scan {time.perf_counter() - t0:.0f} s")
        _check(ids, d, st.ids, st.d2)
        assert np.all(ids[:3, 0] == starts[:3]) and np.all(d[:3, 0] == 0.0)  # exact copies

