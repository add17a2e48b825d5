"""GPU parity at the benchmark sizes, in the benchmark's launch configuration.

* Exact 1-NN ED over 100,000,000 random walks of length 256 (16 segments,
  8-bit symbols, leaves of 2000), queries answered one at a time, a 10-NN
  call over the same queries, the 10-NN classifier's vote, and a screened
  batch (rows equal to single calls; the oracle's queries among them).  The oracle scans the whole collection,
  regenerated on the host in chunks by the seeded generator.
* Exact 1-NN DTW (radius 25) over 10,000,000 random walks of length 256 with
  noisy dataset copies as queries.  For noise 0.01 and 0.1 the oracle's
  LB_Keogh-filtered brute force (equal to the plain scan, pinned on the CPU)
  gives the exact answer; for noise 1.0 that scan is too slow on the host, so
  the answer is checked by properties that hold at any size: its distance is
  the oracle's DTW of the returned series, and no larger than the oracle's
  DTW of the query's source series nor of its ED nearest neighbour.

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


def _say(msg):
    print(f"[scale] {msg}", file=sys.stderr, flush=True)


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
    t0 = time.perf_counter()
    for c in range(0, n, CHUNK):
        raw = synth.randomwalk(min(CHUNK, n - c), length, seed=synth.SEED_DATA, id0=c)
        for st in states:
            st.scan(raw, c)
        if (c // CHUNK) % 10 == 9:
            _say(f"oracle scanned {c + len(raw)} / {n} series ({time.perf_counter() - t0:.0f} s)")


def _check(ids, d, oids, od2):
    assert np.array_equal(ids, oids), (ids, oids)
    od = np.sqrt(od2)
    assert np.all(np.abs(d - od) <= 1e-4 * np.maximum(od, 1e-3)), (d, od)


def test_ed_100m_one_query_at_a_time(pm):
    n, length = 100_000_000, 256
    _say(f"ED: building the index over {n} x {length}")
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    idx = _device_index(pm, n, length, 2000, labels)
    qn, _, _ = synth.noisy_queries(3, n, length)  # noise 0.01, 0.1, 1.0
    qs = np.concatenate([synth.random_queries(3, length), qn[[0, 2]]])
    qt = torch.from_numpy(qs).cuda()
    one = [pm.messi_query(idx, qt[j:j + 1], 1) for j in range(len(qs))]
    ids1 = np.concatenate([o[0].cpu().numpy() for o in one])
    d1 = np.concatenate([o[1].cpu().numpy() for o in one])
    ids10, d10 = (t.cpu().numpy() for t in pm.messi_query(idx, qt, 10))
    cls, cids, _ = pm.messi_classify(idx, labels, 4, qt, 10)  # k-NN classifier, k = 10
    cls, cids = cls.cpu().numpy(), cids.cpu().numpy()
    # a screened batch of 37 (these 5 and 32 noisy copies, k 10 / 3): rows
    # equal to one call per query, and the first 5 checked by the oracle below
    qb = np.concatenate([qs, synth.noisy_queries(32, n, length, j0=1000)[0]])
    qbt = torch.from_numpy(qb).cuda()
    kb = [10] * 5 + [3] * 32
    bids, bd, bst = pm.messi_query_batch(idx, qbt, kb, [0] * 37, [0] * 37, flags=pm.MESSI_SCREEN_BF16,
                                         stats=True)
    bids, bd = bids.cpu().numpy(), bd.cpu().numpy()
    assert bst["screened"] > 0
    for j in range(5, 37, 4):
        sid, sd = pm.messi_query(idx, qbt[j:j + 1], 3)
        assert np.array_equal(bids[j, :3], sid.cpu().numpy()[0]) and np.array_equal(bd[j, :3], sd.cpu().numpy()[0])
    idx.free()
    del labels
    _say("ED: GPU answers ready; oracle scan of the whole collection")
    st = oracle.KnnState(qs, 10)
    _host_scan([st], n, length)
    _check(ids1, d1, st.ids[:, :1], st.d2[:, :1])
    _check(ids10, d10, st.ids, st.d2)
    _check(bids[:5], bd[:5], st.ids, st.d2)
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
    qt = torch.from_numpy(qs).cuda()
    one = [pm.messi_query(idx, qt[j:j + 1], 1, pm.MESSI_DTW, r) for j in range(len(qs))]
    ids = np.concatenate([o[0].cpu().numpy() for o in one])[:, 0]
    d = np.concatenate([o[1].cpu().numpy() for o in one])[:, 0]
    idx.free()
    easy = np.nonzero(sig < 0.5)[0]
    hard = np.nonzero(sig >= 0.5)[0]
    _say("DTW: GPU answers ready; oracle scans")
    st_dtw = oracle.KnnState(qs[easy], 1, oracle.DTW, r, lb_keogh=True)
    st_ed = oracle.KnnState(qs[hard], 1)
    _host_scan([st_dtw, st_ed], n, length)
    _check(ids[easy][:, None], d[easy][:, None], st_dtw.ids, st_dtw.d2)
    # noise 1.0: properties of the returned answer
    zq = oracle.znorm(qs[hard])
    for t, j in enumerate(hard):
        x_ans = oracle.znorm(synth.randomwalk(1, length, seed=synth.SEED_DATA, id0=int(ids[j])))[0]
        d_ans = oracle.dtw2(zq[t], x_ans, r)
        assert abs(d[j] - np.sqrt(d_ans)) <= 1e-4 * max(np.sqrt(d_ans), 1e-3)
        for other in (int(src[j]), int(st_ed.ids[t, 0])):
            x_o = oracle.znorm(synth.randomwalk(1, length, seed=synth.SEED_DATA, id0=other))[0]
            assert d_ans <= oracle.dtw2(zq[t], x_o, r)


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

