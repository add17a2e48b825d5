"""GPU tests of the serving loop (messi_server_*): requests mixing ED and DTW
(windows 5, 10 and 20% of the length), k 1 and 10, and noise 0.01 / 0.1 /
1.0, arriving in a burst and then as a Poisson stream, answered by
concurrent continuous batches.  Each result must equal, id for id and bit
for bit, the answer of messi_query for that request alone, and the oracle's
(ids exact, distances within 1e-4 relative)."""
import threading
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, LEN = 40_000, 256


@pytest.fixture(scope="module")
def pm():
    import paper_2110_07519_amd as pm

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pm.lib()
    return pm


@pytest.fixture(scope="module")
def data():
    return synth.randomwalk(N, LEN, seed=41)


@pytest.fixture(scope="module")
def index(pm, data):
    idx = pm.messi_build(torch.from_numpy(data).cuda(), 16, 256, 500)
    yield idx
    idx.free()


def _requests(nreq):
    qs, _, _ = synth.noisy_queries(nreq, N, LEN, data_seed=41)
    rng = np.random.default_rng(synth.SEED_MIX)
    dist = rng.integers(0, 2, nreq)
    win = np.where(dist == 1, rng.choice([12, 25, 51], nreq), 0)
    ks = rng.choice([1, 10], nreq)
    return qs, [int(x) for x in ks], [int(x) for x in dist], [int(x) for x in win]


def _collect(srv, nreq, timeout_s=120):
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < nreq and time.time() < t_end:
        for rid, status, ids, d, lat in srv.poll(256, timeout_ms=50):
            got[rid] = (status, ids, d, lat)
    assert len(got) == nreq
    return got


def _alone(pm, idx, q, k, dist, win):
    ids, d = pm.messi_query(idx, torch.from_numpy(q[None, :]).cuda(), k, dist, win)
    return ids.cpu().numpy()[0], d.cpu().numpy()[0]


def test_mixed_stream_equals_single_queries(pm, index, data):
    nreq = 90
    qs, ks, dist, win = _requests(nreq)
    srv = pm.Server(index, workers=2, max_batch=64, flags=pm.MESSI_SCREEN_BF16, kmax=10)
    ids_of = {}

    def producer():
        rng = np.random.default_rng(synth.SEED_ARRIVAL)
        for i in range(nreq):
            if i >= 30:  # a burst, then Poisson arrivals (mean gap 0.5 ms)
                time.sleep(rng.exponential(0.0005))
            ids_of[srv.submit(qs[i], ks[i], dist[i], win[i])] = i

    th = threading.Thread(target=producer)
    th.start()
    got = _collect(srv, nreq)
    th.join()
    st = srv.stats()
    srv.stop()
    assert st["completed"] == nreq and st["batches"] < nreq
    for rid, (status, ids, d, lat) in got.items():
        i = ids_of[rid]
        assert status == 0 and lat > 0
        a_ids, a_d = _alone(pm, index, qs[i], ks[i], dist[i], win[i])
        assert np.array_equal(ids[:ks[i]], a_ids) and np.array_equal(d[:ks[i]], a_d)
        assert np.all(ids[ks[i]:] == -1)
    # the oracle on a sample of the mix
    for i in range(0, nreq, 9):
        oids, od2 = oracle.knn(data, qs[i:i + 1], ks[i], distance=dist[i], r=win[i])
        rid = [r for r, j in ids_of.items() if j == i][0]
        _, ids, d, _ = got[rid]
        assert np.array_equal(ids[:ks[i]], oids[0])
        od = np.sqrt(od2[0])
        assert np.all(np.abs(d[:ks[i]] - od) <= 1e-4 * np.maximum(od, 1e-3))


def test_memory_admission_bounds_inflight_requests(pm, index):
    """Every worker holds the buffers of its batch capacity from the start;
    the capacity is cut until all workers fit the budget, and admitted
    requests never hold more than it."""
    nreq = 40
    qs, ks, dist, win = _requests(nreq)
    probe = pm.Server(index, workers=1, max_batch=8, kmax=10)
    per = probe.stats()["request_bytes"]
    probe.stop()
    budget = 8 * per
    srv = pm.Server(index, workers=2, max_batch=64, mem_budget_bytes=budget, kmax=10)
    st0 = srv.stats()
    assert 1 <= st0["batch_capacity"] <= 4 and st0["resident_bytes"] <= budget
    ids_of = {srv.submit(qs[i], ks[i], dist[i], win[i]): i for i in range(nreq)}
    got = _collect(srv, nreq)
    st = srv.stats()
    srv.stop()
    assert st["completed"] == nreq
    assert st["max_batch_seen"] <= st["batch_capacity"]
    # a batch whose near-tie log grew was charged the growth while it ran
    assert st["peak_inflight_bytes"] <= budget + st["log_growth_bytes"] and st["inflight_bytes"] == 0
    assert st["resident_bytes"] == st0["resident_bytes"]
    for rid, (status, ids, d, _) in got.items():
        i = ids_of[rid]
        a_ids, a_d = _alone(pm, index, qs[i], ks[i], dist[i], win[i])
        assert status == 0
        assert np.array_equal(ids[:ks[i]], a_ids) and np.array_equal(d[:ks[i]], a_d)


def test_near_tie_log_growth_is_charged_and_returned(pm, index, data):
    """A flat query (z-normalised to zeros) is at the same distance from
    every series, so all 40,000 are near ties: its near-tie log overflows
    and grows twice (4,096 -> 16,384 -> 65,536 entries).  The growth is
    charged to the in-flight bytes while the batch runs and handed back
    with the memory once the log is shrunk after it."""
    srv = pm.Server(index, workers=1, max_batch=4, kmax=5)
    st0 = srv.stats()
    flat = np.full(LEN, 3.0, np.float32)
    rid = srv.submit(flat, 5)
    got = _collect(srv, 1)
    st = srv.stats()
    srv.stop()
    status, ids, d, _ = got[rid]
    assert status == 0
    a_ids, a_d = _alone(pm, index, flat, 5, 0, 0)
    assert np.array_equal(ids[:5], a_ids) and np.array_equal(d[:5], a_d)
    oids, od2 = oracle.knn(data, flat[None, :], 5)
    assert np.array_equal(ids[:5], oids[0])
    grown = (65536 - 4096) * 8  # log bytes added for one query slot (at least)
    assert st["log_growth_bytes"] >= grown
    assert st["peak_inflight_bytes"] >= st0["request_bytes"] + grown
    assert st["inflight_bytes"] == 0
    assert st["resident_bytes"] == st0["resident_bytes"]


def test_server_argument_errors(pm, index):
    srv = pm.Server(index, workers=1, max_batch=4, kmax=5)
    q = synth.random_queries(1, LEN)[0]
    with pytest.raises(pm.MessiError):
        srv.submit(q, 6)
    with pytest.raises(pm.MessiError):
        srv.submit(q, 1, 3)
    with pytest.raises(pm.MessiError):
        srv.submit(q, 1, 1, -2)
    srv.stop()
    with pytest.raises(pm.MessiError):
        pm.Server(index, workers=9)
