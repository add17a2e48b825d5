"""GPU parity of batched queries (messi_query_batch): per-query k, distance
and window in one call, with and without the BF16 MFMA screen, against the
CPU oracle (ids exact, distances within 1e-4 relative) and against one call
per query (identical ids and distances)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pm():
    import paper_2110_07519_amd as pm

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pm.lib()
    return pm


def _oracle_rows(raw, qs, ks, dist, win):
    """Expected (ids, d) per query from the brute-force oracle, padded to kmax."""
    kmax = int(max(ks))
    ids = np.full((len(qs), kmax), -1, dtype=np.int64)
    d = np.full((len(qs), kmax), np.inf)
    for key in sorted(set(zip(dist, win))):
        sel = [i for i in range(len(qs)) if (dist[i], win[i]) == key]
        kk = max(ks[i] for i in sel)
        oi, od2 = oracle.knn(raw, qs[sel], kk, distance=key[0], r=key[1])
        for t, i in enumerate(sel):
            ids[i, :ks[i]] = oi[t, :ks[i]]
            d[i, :ks[i]] = np.sqrt(od2[t, :ks[i]])
    return ids, d


def _check(ids, d, oids, od):
    assert np.array_equal(ids, oids), np.nonzero((ids != oids).any(axis=1))[0]
    fin = np.isfinite(od)
    assert np.array_equal(np.isfinite(d), fin)
    assert np.all(np.abs(d[fin] - od[fin]) <= 1e-4 * np.maximum(od[fin], 1e-3))


def _run(pm, idx, qt, ks, dist, win, flags):
    ids, d, st = pm.messi_query_batch(idx, qt, ks, dist, win, flags=flags, stats=True)
    return ids.cpu().numpy(), d.cpu().numpy(), st


@pytest.mark.parametrize("length", [256, 128, 64])
def test_mixed_batch_matches_oracle_and_single_calls(pm, length):
    n = 30_000
    raw = synth.randomwalk(n, length, seed=31)
    raw = np.concatenate([raw, raw[:200]])  # exact duplicates: ties
    qn, _, _ = synth.noisy_queries(60, n, length, data_seed=31)
    qs = np.concatenate([qn, synth.random_queries(6, length), raw[[3, 150]]])
    nq = len(qs)
    rng = np.random.default_rng(4)
    ks = [1 if i % 2 == 0 else 10 for i in range(nq)]
    dist = [0 if i % 3 else 1 for i in range(nq)]
    wins = [int(rng.choice([0, 3, length // 10])) if dist[i] == 1 else 0 for i in range(nq)]
    t = torch.from_numpy(raw).cuda()
    idx = pm.messi_build(t, 16, 256, 500)
    qt = torch.from_numpy(qs).cuda()
    oids, od = _oracle_rows(raw, qs, ks, dist, wins)
    plain = _run(pm, idx, qt, ks, dist, wins, 0)
    _check(plain[0], plain[1], oids, od)
    scr = _run(pm, idx, qt, ks, dist, wins, pm.MESSI_SCREEN_BF16)
    _check(scr[0], scr[1], oids, od)
    assert np.array_equal(plain[0], scr[0]) and np.array_equal(plain[1], scr[1])
    assert scr[2]["screened"] > 0
    # one call per query gives the same rows
    for i in range(0, nq, 7):
        ids1, d1 = pm.messi_query(idx, qt[i:i + 1], ks[i], dist[i], wins[i])
        assert np.array_equal(ids1.cpu().numpy()[0], plain[0][i, :ks[i]])
        assert np.array_equal(d1.cpu().numpy()[0], plain[1][i, :ks[i]])
    idx.free()


def test_screen_with_many_ties_and_large_k(pm):
    base = synth.randomwalk(3000, 128, seed=5)
    raw = np.concatenate([base, np.repeat(base[7:8], 2500, axis=0)])
    t = torch.from_numpy(raw).cuda()
    idx = pm.messi_build(t, 16, 256, 100)
    qs = np.concatenate([raw[[7, 11, 2999]], synth.noisy_queries(29, 3000, 128, data_seed=5)[0]])
    qt = torch.from_numpy(qs).cuda()
    ks = ([3, 50, 1, 64, 2, 7, 1, 20] * 4)[:len(qs)]
    oids, od = _oracle_rows(raw, qs, ks, [0] * len(qs), [0] * len(qs))
    for flags in (0, pm.MESSI_SCREEN_BF16):
        ids, d, _ = _run(pm, idx, qt, ks, [0] * len(qs), [0] * len(qs), flags)
        _check(ids, d, oids, od)
    idx.free()


def test_screen_ignored_for_unsupported_length(pm):
    raw96 = synth.randomwalk(4000, 96, seed=9)    # the screen serves 64, 128, 256, 512 only
    raw100 = synth.randomwalk(4000, 100, seed=9)
    for data in (raw96, raw100):
        length = data.shape[1]
        t = torch.from_numpy(data).cuda()
        idx = pm.messi_build(t, 4 if length == 100 else 16, 256, 50)
        qs = synth.noisy_queries(40, 4000, length, data_seed=9)[0]
        qt = torch.from_numpy(qs).cuda()
        ks = [1, 5, 2, 1, 3, 1, 4, 2] * 5
        oids, od = _oracle_rows(data, qs, ks, [0] * 40, [0] * 40)
        ids, d, st = _run(pm, idx, qt, ks, [0] * 40, [0] * 40, pm.MESSI_SCREEN_BF16)
        assert st["screened"] == 0
        _check(ids, d, oids, od)
        idx.free()


def test_batch_edge_cases_and_errors(pm):
    raw = synth.randomwalk(6, 64, seed=2)
    t = torch.from_numpy(raw).cuda()
    idx = pm.messi_build(t, 16, 256, 2)
    qs = synth.random_queries(3, 64)
    qt = torch.from_numpy(qs).cuda()
    ids, d = pm.messi_query_batch(idx, qt, [8, 1, 3], [0, 0, 1], [0, 0, 5], kmax=9,
                                  flags=pm.MESSI_SCREEN_BF16)
    ids, d = ids.cpu().numpy(), d.cpu().numpy()
    oids, od = _oracle_rows(raw, qs, [8, 1, 3], [0, 0, 1], [0, 0, 5])
    pad = np.full((3, 1), -1), np.full((3, 1), np.inf)
    _check(ids, d, np.concatenate([oids, pad[0]], axis=1), np.concatenate([od, pad[1]], axis=1))
    e = torch.empty((0, 64), dtype=torch.float32, device="cuda")
    o1, _ = pm.messi_query_batch(idx, e, [], [], [], kmax=2)
    assert o1.shape == (0, 2)
    with pytest.raises(pm.MessiError):
        pm.messi_query_batch(idx, qt, [3, 1, 1], [0, 0, 0], [0, 0, 0], kmax=2)
    with pytest.raises(pm.MessiError):
        pm.messi_query_batch(idx, qt, [1, 1, 1], [0, 2, 0], [0, 0, 0])
    with pytest.raises(pm.MessiError):
        pm.messi_query_batch(idx, qt, [1, 1, 1], [1, 1, 1], [0, -1, 0])
    with pytest.raises(pm.MessiError):
        pm.messi_query_batch(idx, qt, [1, 1, 1], [0, 0, 0], [0, 0, 0], flags=8)
    idx.free()


def test_screen_length_512(pm):
    raw = synth.randomwalk(5000, 512, seed=12)
    t = torch.from_numpy(raw).cuda()
    idx = pm.messi_build(t, 16, 256, 100)
    qs = np.concatenate([synth.noisy_queries(33, 5000, 512, data_seed=12)[0],
                         synth.random_queries(3, 512)])
    qt = torch.from_numpy(qs).cuda()
    ks = [1, 10] * 18
    oids, od = _oracle_rows(raw, qs, ks, [0] * 36, [0] * 36)
    for flags in (0, pm.MESSI_SCREEN_BF16):
        ids, d, st = _run(pm, idx, qt, ks, [0] * 36, [0] * 36, flags)
        _check(ids, d, oids, od)
    assert st["screened"] > 0
    idx.free()
