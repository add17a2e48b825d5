"""GPU tests of how batches run: overlapped (distance, window) groups, HIP
graph capture and replay (MESSI_GRAPH), the autotuner and its JSON cache,
the index memory budget, and an in-place store the index takes over.
Answers are checked against the CPU oracle (ids exact, distances within
1e-4 relative) and, bit for bit, against the eager path."""
import ctypes
import json

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, LEN = 20_000, 256


@pytest.fixture(scope="module")
def pm():
    import paper_2110_07519_amd as pm

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pm.lib()
    return pm


@pytest.fixture(scope="module")
def data():
    return synth.randomwalk(N, LEN, seed=51)


@pytest.fixture(scope="module")
def index(pm, data):
    idx = pm.messi_build(torch.from_numpy(data).cuda(), 16, 256, 400)
    pm.messi_prepare_screen(idx)
    yield idx
    idx.free()


def _mix(nq, seed):
    """nq noisy copies; ED (k 1 / 10) and DTW with r 5 and 25 (k 3)."""
    qs, _, _ = synth.noisy_queries(nq, N, LEN, data_seed=51, j0=seed)
    dist = [0 if i % 3 else 1 for i in range(nq)]
    win = [0 if dist[i] == 0 else (5 if i % 2 else 25) for i in range(nq)]
    ks = [(1 if i % 2 else 10) if dist[i] == 0 else 3 for i in range(nq)]
    return qs, ks, dist, win


def _oracle_rows(raw, qs, ks, dist, win, kmax):
    ids = np.full((len(qs), kmax), -1, dtype=np.int64)
    d = np.full((len(qs), kmax), np.inf)
    for key in sorted(set(zip(dist, win))):
        sel = [i for i in range(len(qs)) if (dist[i], win[i]) == key]
        oi, od2 = oracle.knn(raw, qs[sel], max(ks[i] for i in sel), distance=key[0], r=key[1])
        for t, i in enumerate(sel):
            ids[i, :ks[i]] = oi[t, :ks[i]]
            d[i, :ks[i]] = np.sqrt(od2[t, :ks[i]])
    return ids, d


def _check(ids, d, oids, od):
    assert np.array_equal(ids, oids), np.nonzero((ids != oids).any(axis=1))[0]
    fin = np.isfinite(od)
    assert np.array_equal(np.isfinite(d), fin)
    assert np.all(np.abs(d[fin] - od[fin]) <= 1e-4 * np.maximum(od[fin], 1e-3))


def _host(t):
    return t.cpu().numpy()


def test_overlapped_groups_match_oracle_and_single_calls(pm, index, data):
    """A batch of three (distance, window) groups runs them concurrently on
    their own streams; every row equals the oracle's and messi_query's."""
    qs, ks, dist, win = _mix(45, 7000)
    qt = torch.from_numpy(qs).cuda()
    ids, d, st = pm.messi_query_batch(index, qt, ks, dist, win, kmax=10, flags=pm.MESSI_SCREEN_BF16,
                                      stats=True)
    ids, d = _host(ids), _host(d)
    assert st["queries"] == 45
    _check(ids, d, *_oracle_rows(data, qs, ks, dist, win, 10))
    for i in range(0, 45, 4):
        a_ids, a_d = pm.messi_query(index, qt[i:i + 1], ks[i], dist[i], win[i])
        assert np.array_equal(ids[i, :ks[i]], _host(a_ids)[0]) and np.array_equal(d[i, :ks[i]], _host(a_d)[0])
    # the same batch without statistics (no phase events) gives the same rows
    ids2, d2 = pm.messi_query_batch(index, qt, ks, dist, win, kmax=10, flags=pm.MESSI_SCREEN_BF16)
    assert np.array_equal(ids, _host(ids2)) and np.array_equal(d, _host(d2))


@pytest.mark.parametrize("mixed", [False, True])
def test_graph_replays_equal_eager_calls(pm, index, data, mixed):
    """MESSI_GRAPH: the first call captures the batch, later calls with the
    same launches replay it.  The query buffer is refilled between replays
    (a replay reads the buffer's current contents) and other work runs on
    the device in between; every replay must equal the eager call on the
    same contents, and the oracle."""
    nq = 40
    if mixed:
        qs0, ks, dist, win = _mix(nq, 8000)
    else:
        qs0, _, _ = synth.noisy_queries(nq, N, LEN, data_seed=51, j0=8000)
        ks, dist, win = [1 if i % 2 else 10 for i in range(nq)], [0] * nq, [0] * nq
    flags = pm.MESSI_SCREEN_BF16
    qt = torch.from_numpy(qs0).cuda()
    out_i = torch.empty((nq, 10), dtype=torch.int64, device="cuda")
    out_d = torch.empty((nq, 10), dtype=torch.float32, device="cuda")
    for rep in range(4):
        qs = synth.noisy_queries(nq, N, LEN, data_seed=51, j0=8000 + 100 * rep)[0]
        qt.copy_(torch.from_numpy(qs))
        e_ids, e_d = pm.messi_query_batch(index, qt, ks, dist, win, kmax=10, flags=flags)
        e_ids, e_d = _host(e_ids), _host(e_d)
        pm.messi_query_batch(index, qt, ks, dist, win, kmax=10, flags=flags | pm.MESSI_GRAPH,
                             out_ids=out_i, out_dists=out_d)
        torch.cuda.synchronize()
        g_ids, g_d = _host(out_i), _host(out_d)
        assert np.array_equal(g_ids, e_ids) and np.array_equal(g_d, e_d), rep
        if rep in (0, 3):
            _check(g_ids, g_d, *_oracle_rows(data, qs, ks, dist, win, 10))
        # unrelated device work between replays
        pm.messi_query(index, qt[:2], 4)
        torch.cuda.synchronize()
    # other k: other launches, so a new capture, still equal to eager
    ks2 = [3] * nq
    e_ids, e_d = pm.messi_query_batch(index, qt, ks2, dist, win, kmax=10, flags=flags)
    g_ids, g_d = pm.messi_query_batch(index, qt, ks2, dist, win, kmax=10, flags=flags | pm.MESSI_GRAPH)
    assert np.array_equal(_host(g_ids), _host(e_ids)) and np.array_equal(_host(g_d), _host(e_d))


def test_autotune_cache_round_trip(pm, data, tmp_path):
    cache = str(tmp_path / "tune.json")
    t = torch.from_numpy(data).cuda()
    idx = pm.messi_build_ex(t, 16, 256, 400, bf16_screen=True, autotune_cache=cache)
    qs, ks, dist, win = _mix(48, 9000)
    qt = torch.from_numpy(qs).cuda()
    before = pm.messi_query_batch(idx, qt, ks, dist, win, kmax=10, flags=pm.MESSI_SCREEN_BF16)
    tune = pm.messi_autotune(idx, qt, ks, dist, win, kmax=10, flags=pm.MESSI_SCREEN_BF16)
    assert tune["from_cache"] == 0 and tune["candidates"] >= 2 and tune["ms"] > 0
    assert tune["ms"] <= tune["ms_default"]
    entries = json.load(open(cache))
    assert len(entries) == 1
    (key, val), = entries.items()
    assert "/nq64/" in key and "dtw25" in key and "dtw5" in key and key.endswith("/screen")
    for name in ("screen", "screen_nt", "screen_occ", "ed_scale", "dtw_scale", "overlap"):
        assert val[name] == tune[name]
    # tuned knobs give the same answers
    after = pm.messi_query_batch(idx, qt, ks, dist, win, kmax=10, flags=pm.MESSI_SCREEN_BF16)
    assert all(np.array_equal(_host(a), _host(b)) for a, b in zip(before, after))
    assert pm.messi_autotune(idx, qt, ks, dist, win, kmax=10, flags=pm.MESSI_SCREEN_BF16)["from_cache"] == 1
    idx.free()
    # a new index reads the file: the same shape is a cache hit
    idx2 = pm.messi_build_ex(t, 16, 256, 400, bf16_screen=True, autotune_cache=cache)
    again = pm.messi_autotune(idx2, qt, ks, dist, win, kmax=10, flags=pm.MESSI_SCREEN_BF16)
    assert again["from_cache"] == 1 and again["screen_nt"] == tune["screen_nt"]
    # a second shape (ED only, no screen) adds an entry and keeps the first
    e = pm.messi_autotune(idx2, qt[:20], 1, 0, 0, kmax=1)
    assert e["from_cache"] == 0
    assert len(json.load(open(cache))) == 2
    idx2.free()
    # a file this library did not write is refused
    bad = tmp_path / "bad.json"
    bad.write_text("[1, 2, 3]")
    with pytest.raises(pm.MessiError) as err:
        pm.messi_build_ex(t, 16, 256, 400, autotune_cache=str(bad))
    assert err.value.code == pm.MESSI_EINVAL


def test_memory_budget(pm, data):
    t = torch.from_numpy(data).cuda()
    with pytest.raises(pm.MessiError) as err:
        pm.messi_build_ex(t, 16, 256, 400, mem_budget_bytes=1 << 20)  # less than the copy
    assert err.value.code == pm.MESSI_ENOMEM
    free = pm.messi_build(t, 16, 256, 400)
    held = pm.messi_index_info(free)["device_bytes"]
    free.free()
    budget = held + (8 << 20)
    idx = pm.messi_build_ex(t, 16, 256, 400, mem_budget_bytes=budget)
    q = torch.from_numpy(synth.random_queries(4, LEN)).cuda()
    ids, d = pm.messi_query(idx, q, 3)  # a small workspace fits
    oids, od2 = oracle.knn(data, synth.random_queries(4, LEN), 3)
    _check(_host(ids), _host(d), oids, np.sqrt(od2))
    assert pm.messi_index_info(idx)["device_bytes"] <= budget
    with pytest.raises(pm.MessiError) as err:  # the BF16 copy (2 bytes a value) does not
        pm.messi_prepare_screen(idx)
    assert err.value.code == pm.MESSI_ENOMEM
    big = torch.from_numpy(synth.random_queries(2000, LEN)).cuda()
    with pytest.raises(pm.MessiError) as err:  # nor the workspace of 2000 queries
        pm.messi_query(idx, big, 1)
    assert err.value.code == pm.MESSI_ENOMEM
    assert pm.messi_index_info(idx)["device_bytes"] <= budget
    ids2, d2 = pm.messi_query(idx, q, 3)  # and the index still answers
    assert np.array_equal(_host(ids2), _host(ids))
    idx.free()


def test_inplace_store_taken_over(pm):
    """messi_options.inplace = 2: the index z-normalises a hipMalloc'd
    buffer in place and frees it in messi_free."""
    L = pm.lib()  # hipMalloc / hipMemcpy / hipFree / hipMemGetInfo of the library's HIP runtime
    L.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    L.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    L.hipFree.argtypes = [ctypes.c_void_p]
    L.hipMemGetInfo.argtypes = [ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    n = 240_000  # a 245 MB store: its release shows in the free memory
    raw = synth.randomwalk(n, LEN, seed=52)
    nbytes = raw.nbytes
    ptr = ctypes.c_void_p()
    assert L.hipMalloc(ctypes.byref(ptr), nbytes) == 0
    assert L.hipMemcpy(ptr, raw.ctypes.data_as(ctypes.c_void_p), nbytes, 1) == 0
    # not the start of the allocation: refused, nothing taken
    with pytest.raises(pm.MessiError) as err:
        pm.messi_build_owned(ptr.value + 4 * LEN, raw.shape[0] - 1, LEN, leaf_size=400)
    assert err.value.code == pm.MESSI_EINVAL
    idx = pm.messi_build_owned(ptr.value, raw.shape[0], LEN, leaf_size=400)
    qs = synth.noisy_queries(6, n, LEN, data_seed=52)[0]
    ids, d = pm.messi_query(idx, torch.from_numpy(qs).cuda(), 2)
    oids, od2 = oracle.knn(raw, qs, 2)
    _check(_host(ids), _host(d), oids, np.sqrt(od2))
    torch.cuda.synchronize()
    f0, f1, tot = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    assert L.hipMemGetInfo(ctypes.byref(f0), ctypes.byref(tot)) == 0
    idx.free()  # frees the store too
    assert L.hipMemGetInfo(ctypes.byref(f1), ctypes.byref(tot)) == 0
    assert f1.value - f0.value >= nbytes


def test_ed_batch_larger_than_the_process_grid(pm, index, data):
    """An unscreened ED batch of more queries than the process kernel has
    blocks (its grid is one resident wave of blocks, a few hundred): every
    query's approximate-search candidates must still reach its near-tie log
    (they are skipped by the leaf pass), so each row equals a single call's
    and the oracle's."""
    nq = 1100
    qs, _, _ = synth.noisy_queries(nq, N, LEN, data_seed=51, j0=12000)
    ks = [1 if i % 2 == 0 else 5 for i in range(nq)]
    qt = torch.from_numpy(qs).cuda()
    ids, d = (_host(t) for t in pm.messi_query_batch(index, qt, ks, 0, 0, kmax=5))
    for i in range(nq):
        a_ids, a_d = pm.messi_query(index, qt[i:i + 1], ks[i])
        assert np.array_equal(ids[i, :ks[i]], _host(a_ids)[0]) and np.array_equal(d[i, :ks[i]], _host(a_d)[0]), i
    assert np.all(ids[0::2, 1:] == -1)
    oids, od2 = oracle.knn(data, qs, 5)
    for i in range(nq):
        _check(ids[i:i + 1, :ks[i]], d[i:i + 1, :ks[i]], oids[i:i + 1, :ks[i]], np.sqrt(od2[i:i + 1, :ks[i]]))


def test_screen_lists_longer_than_the_lds_copy(pm):
    """A screened batch of 2,300 queries over 4,000 series in leaves of up
    to 400: most leaves are kept by more queries than the screen stages in
    LDS (2,048), so their lists are read from memory.  Rows equal the
    unscreened batch's and the oracle's."""
    raw = synth.randomwalk(4000, LEN, seed=53)
    idx = pm.messi_build(torch.from_numpy(raw).cuda(), 16, 256, 400)
    nq = 2300
    qs = np.concatenate([synth.noisy_queries(nq // 2, 4000, LEN, data_seed=53)[0],
                         synth.random_queries(nq - nq // 2, LEN, seed=54)])
    ks = [1 if i % 3 else 4 for i in range(nq)]
    qt = torch.from_numpy(qs).cuda()
    plain = [_host(t) for t in pm.messi_query_batch(idx, qt, ks, 0, 0, kmax=4)]
    ids, d, st = pm.messi_query_batch(idx, qt, ks, 0, 0, kmax=4, flags=pm.MESSI_SCREEN_BF16, stats=True)
    assert st["screened"] > 0
    assert np.array_equal(_host(ids), plain[0]) and np.array_equal(_host(d), plain[1])
    oids, od2 = oracle.knn(raw, qs, 4)
    for i in range(0, nq, 7):
        _check(plain[0][i:i + 1, :ks[i]], plain[1][i:i + 1, :ks[i]], oids[i:i + 1, :ks[i]],
               np.sqrt(od2[i:i + 1, :ks[i]]))
    idx.free()
