"""GPU parity of the non-normalised index (series and queries as given) and of
subsequence search over sliding windows (messi_build_windows), against the
CPU oracle in its matching mode: words and the leaf partition bitwise,
k-NN ids exactly, distances within 1e-4 relative."""
import contextlib

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


def _check(ids, d, oids, od2):
    assert np.array_equal(ids, oids), (np.nonzero((ids != oids).any(axis=1))[0], ids[:3], oids[:3])
    od = np.sqrt(od2)
    fin = np.isfinite(od)
    assert np.array_equal(np.isfinite(d), fin)
    assert np.all(np.abs(d[fin] - od[fin]) <= 1e-4 * np.maximum(od[fin], 1e-3))


def _offset_rows(n, length, seed, scale=0.05):
    """Random walks with per-row offsets and gains, then scaled so the raw
    values straddle the breakpoints (symbols spread over many leaves)."""
    x = synth.randomwalk(n, length, seed=seed).astype(np.float64)
    rng = np.random.default_rng(seed)
    x = x * rng.uniform(0.3, 3.0, (n, 1)) + rng.uniform(-20.0, 20.0, (n, 1))
    return (x * scale).astype(np.float32)


def _query(pm, idx, qs, k, distance=0, window=0):
    qt = torch.from_numpy(np.ascontiguousarray(qs)).cuda()
    ids, d = pm.messi_query(idx, qt, k, distance, window)
    return ids.cpu().numpy(), d.cpu().numpy()


@pytest.mark.parametrize("n,length,leaf", [(20_000, 256, 200), (1003, 64, 30), (517, 192, 25)])
def test_raw_build_matches_oracle(pm, n, length, leaf):
    raw = _offset_rows(n, length, seed=21)
    raw[5] = 3.0  # a flat row stays as it is in raw mode
    t = torch.from_numpy(raw).cuda()
    idx = pm.messi_build_ex(t, 16, 256, leaf, raw=True)
    with oracle.raw_mode():
        Wo = oracle.words(raw)
    W = pm.messi_get_words(idx)
    assert np.array_equal(W, Wo), np.argwhere(W != Wo)[:5]
    perm, leaves = oracle.leaf_partition(Wo, leaf)
    assert np.array_equal(pm.messi_get_perm(idx), perm)
    gl = pm.messi_get_leaves(idx)
    assert np.array_equal(gl["begin"], leaves["begin"]) and np.array_equal(gl["end"], leaves["end"])
    assert np.array_equal(t.cpu().numpy().view(np.uint32), raw.view(np.uint32))  # only read
    idx.free()


@pytest.mark.parametrize("length", [256, 128])
def test_raw_knn_ed_and_dtw_match_oracle(pm, length):
    n = 30_000
    raw = _offset_rows(n, length, seed=23)
    raw = np.concatenate([raw, raw[:50]])  # exact duplicates: ties
    rng = np.random.default_rng(5)
    src = rng.integers(0, n, 24)
    noisy = raw[src] + rng.normal(0.0, 0.05, (24, length)).astype(np.float32)
    qs = np.concatenate([noisy, _offset_rows(4, length, seed=24), raw[[7, 20_001]]]).astype(np.float32)
    t = torch.from_numpy(raw).cuda()
    idx = pm.messi_build_ex(t, 16, 256, 500, raw=True)
    with oracle.raw_mode():
        for k in (1, 10):
            oids, od2 = oracle.knn(raw, qs, k)
            _check(*_query(pm, idx, qs, k), oids, od2)
        for r in (3, length // 10):
            oids, od2 = oracle.knn(raw, qs[:12], 5, distance=oracle.DTW, r=r)
            _check(*_query(pm, idx, qs[:12], 5, 1, r), oids, od2)
    idx.free()


def test_raw_inplace_and_batch_screen(pm):
    n, length = 25_000, 128
    raw = _offset_rows(n, length, seed=27)
    rng = np.random.default_rng(6)
    qs = (raw[rng.integers(0, n, 40)] + rng.normal(0.0, 0.1, (40, length))).astype(np.float32)
    t = torch.from_numpy(raw.copy()).cuda()
    idx = pm.messi_build_ex(t, 16, 256, 300, inplace=True, raw=True)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy().view(np.uint32), raw.view(np.uint32))  # rows untouched
    with oracle.raw_mode():
        oids, od2 = oracle.knn(raw, qs, 3)
    _check(*_query(pm, idx, qs, 3), oids, od2)
    qt = torch.from_numpy(qs).cuda()
    ks, dist, win = [3] * 40, [0] * 40, [0] * 40
    for flags in (0, pm.MESSI_SCREEN_BF16):
        ids, d, st = pm.messi_query_batch(idx, qt, ks, dist, win, flags=flags, stats=True)
        _check(ids.cpu().numpy(), d.cpu().numpy(), oids, od2)
    assert st["screened"] > 0
    idx.free()


def _long_series(total, seed):
    return synth.randomwalk(1, total, seed=seed)[0] * np.float32(0.1)


@pytest.mark.parametrize("length,stride,as_given", [(128, 1, True), (256, 5, True), (64, 3, False)])
def test_windows_match_oracle(pm, length, stride, as_given):
    total = 200_000
    s = _long_series(total, seed=31)
    st = torch.from_numpy(s).cuda()
    idx = pm.messi_build_windows(st, length, stride, leaf_size=400, raw=as_given)
    Wd = oracle.windows(s, length, stride)
    assert idx.n == len(Wd) == (total - length) // stride + 1
    rng = np.random.default_rng(length + stride)
    starts = rng.integers(0, total - length, 16)
    qs = np.stack([s[a:a + length] for a in starts])
    qs[8:] += rng.normal(0.0, 0.02, (8, length)).astype(np.float32)
    mode = oracle.raw_mode() if as_given else contextlib.nullcontext()
    with mode:
        Wo = oracle.words(Wd)
        oids, od2 = oracle.knn(Wd, qs, 5)
        dids, dd2 = oracle.knn(Wd, qs[:6], 2, distance=oracle.DTW, r=length // 20)
    assert np.array_equal(pm.messi_get_words(idx), Wo)
    ids, d = _query(pm, idx, qs, 5)
    _check(ids, d, oids, od2)
    _check(*_query(pm, idx, qs[:6], 2, 1, length // 20), dids, dd2)
    # an exact copy of a window is found at that window's start
    for j in range(8):
        if starts[j] % stride == 0:
            assert ids[j, 0] == starts[j] // stride and d[j, 0] == 0.0
    assert np.array_equal(st.cpu().numpy().view(np.uint32), s.view(np.uint32))  # only read
    idx.free()


def test_windows_edges_and_errors(pm):
    s = _long_series(320, seed=33)
    st = torch.from_numpy(s).cuda()
    one = pm.messi_build_windows(st, 320, 1, leaf_size=4)  # a single window
    assert one.n == 1
    ids, d = _query(pm, one, s[None, :], 1)
    assert ids[0, 0] == 0 and d[0, 0] == 0.0
    one.free()
    ragged = pm.messi_build_windows(st, 64, 7, leaf_size=4)  # the tail shorter than a stride
    Wd = oracle.windows(s, 64, 7)
    assert ragged.n == len(Wd) == 37
    with oracle.raw_mode():
        oids, od2 = oracle.knn(Wd, Wd[[0, 36]], 3)
    _check(*_query(pm, ragged, Wd[[0, 36]], 3), oids, od2)
    ragged.free()
    for bad in [dict(length=321, stride=1), dict(length=64, stride=0), dict(length=0, stride=1),
                dict(length=60, stride=1, segments=16)]:
        with pytest.raises(pm.MessiError):
            pm.messi_build_windows(st, **bad)
