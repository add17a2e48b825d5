"""GPU parity: the HIP library against the CPU oracle, element by element, on
the same seeded inputs.  Words, the leaf-order permutation and the leaf
table are compared bitwise; k-NN ids exactly; distances within 1e-4
relative (|d - d64| <= 1e-4 max(d64, 1e-3))."""
import os

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


def _build(pm, raw, segments=16, cardinality=256, leaf_size=2000):
    t = torch.from_numpy(np.ascontiguousarray(raw)).cuda()
    idx = pm.messi_build(t, segments, cardinality, leaf_size)
    return idx, t


def _query(pm, idx, qs, k, distance=0, window=0, stats=False):
    qt = torch.from_numpy(np.ascontiguousarray(qs)).cuda()
    out = pm.messi_query(idx, qt, k, distance, window, stats=stats)
    ids = out[0].cpu().numpy()
    d = out[1].cpu().numpy()
    return (ids, d, out[2]) if stats else (ids, d)


def _check_answers(ids, d, oids, od2):
    assert np.array_equal(ids, oids), (np.nonzero((ids != oids).any(axis=1))[0], ids[:3], oids[:3])
    od = np.sqrt(od2)
    fin = np.isfinite(od)
    assert np.all(np.isfinite(d) == fin)
    assert np.all(np.abs(d[fin] - od[fin]) <= 1e-4 * np.maximum(od[fin], 1e-3))


def test_device_generator_matches_host():
    for count, length in [(10_000, 256), (1001, 128), (65, 100), (130, 1024)]:
        t = torch.empty((count, length), dtype=torch.float32, device="cuda")
        synth.randomwalk_device(t, seed=1, id0=7)
        torch.cuda.synchronize()
        h = synth.randomwalk(count, length, seed=1, id0=7)
        assert np.array_equal(t.cpu().numpy().view(np.uint32), h.view(np.uint32))


@pytest.mark.parametrize("n,length,w,card,leaf", [
    (100_000, 256, 16, 256, 2000),   # the tiny configuration
    (3001, 128, 16, 256, 50),        # ragged tail, deep splits
    (1003, 64, 16, 256, 30),         # 4 points per segment
    (517, 192, 16, 16, 25),          # 12 points per segment, 4-bit symbols
    (777, 96, 8, 16, 20),            # fewer segments, 4-bit symbols
    (500, 100, 4, 4, 7),             # length not a multiple of 4
    (300, 16, 16, 2, 5),             # one point per segment, 1-bit symbols (over-full leaves)
])
def test_build_matches_oracle(pm, n, length, w, card, leaf):
    raw = synth.randomwalk(n, length, seed=11)
    raw[3] = 5.0  # a flat series: z-normalised to zeros
    idx, _ = _build(pm, raw, w, card, leaf)
    cb = card.bit_length() - 1
    W = pm.messi_get_words(idx)
    Wo = oracle.words(raw, w, cb)
    assert np.array_equal(W, Wo), np.argwhere(W != Wo)[:5]
    perm, leaves = oracle.leaf_partition(Wo, leaf, cb)
    gperm = pm.messi_get_perm(idx)
    gl = pm.messi_get_leaves(idx)
    assert len(gl) == len(leaves)
    assert np.array_equal(gl["begin"], leaves["begin"]) and np.array_equal(gl["end"], leaves["end"])
    assert np.array_equal(gl["sym"][:, :w], leaves["sym"][:, :w])
    assert np.array_equal(gl["bits"][:, :w], leaves["bits"][:, :w])
    assert np.array_equal(gperm, perm)
    idx.free()


@pytest.mark.parametrize("n,length,w,card,leaf", [
    (3001, 128, 16, 256, 50),
    (1003, 64, 16, 256, 30),
    (517, 192, 16, 16, 25),
    (777, 96, 8, 16, 20),
    (500, 100, 4, 4, 7),
    (300, 16, 16, 2, 5),
    (400, 55, 5, 16, 10),            # length not a multiple of 4: DTW steps one row at a time
])
def test_query_odd_shapes(pm, n, length, w, card, leaf):
    """k-NN on the build shapes above (fewer segments, small alphabets, a
    length not a multiple of 4, over-full leaves) under ED and DTW.  The
    queries add a flat one: z-normalised to zeros, it is at distance 0 from
    the flat series and every other series is a near tie at about
    sqrt(len), so the near-tie log and the FP64 recheck see all of them."""
    raw = synth.randomwalk(n, length, seed=11)
    raw[3] = 5.0
    idx, _ = _build(pm, raw, w, card, leaf)
    qn, _, _ = synth.noisy_queries(6, n, length, data_seed=11)
    flat = np.full((1, length), -2.0, np.float32)
    qs = np.concatenate([qn, synth.random_queries(3, length, seed=12), flat, raw[[3, 9]]])
    for k in (1, 4):
        oids, od2 = oracle.knn(raw, qs, k)
        _check_answers(*_query(pm, idx, qs, k), oids, od2)
    for r in (3, 25, length):
        oids, od2 = oracle.knn(raw, qs, 2, distance=oracle.DTW, r=r)
        _check_answers(*_query(pm, idx, qs, 2, 1, r), oids, od2)
    idx.free()


def test_query_ed_tiny_configuration(pm):
    """100,000 x 256 random walks, 100 random-walk queries, exact 1-NN and
    10-NN under ED against the brute-force scan."""
    raw = synth.randomwalk(100_000, 256)
    qs = synth.random_queries(100, 256)
    idx, _ = _build(pm, raw)
    for k in (1, 10):
        oids, od2 = oracle.knn(raw, qs, k)
        ids, d, st = _query(pm, idx, qs, k, stats=True)
        _check_answers(ids, d, oids, od2)
        assert st["refined"] < 100 * 100_000 * 0.5
    # one query at a time gives the same answers
    for j in range(0, 100, 17):
        ids, d = _query(pm, idx, qs[j:j + 1], 1)
        oids, od2 = oracle.knn(raw, qs[j:j + 1], 1)
        _check_answers(ids, d, oids, od2)
    idx.free()


def test_query_ed_noisy_and_exact_copies(pm):
    n = 50_000
    raw = synth.randomwalk(n, 256)
    raw = np.concatenate([raw, raw[:300], raw[:300]])  # exact duplicates: ties on distance
    qn, src, sig = synth.noisy_queries(30, n, 256)
    qs = np.concatenate([qn, raw[[5, 17, 299, 1000]]])
    idx, _ = _build(pm, raw)
    for k in (1, 5):
        oids, od2 = oracle.knn(raw, qs, k)
        ids, d = _query(pm, idx, qs, k)
        _check_answers(ids, d, oids, od2)
    idx.free()


@pytest.mark.parametrize("length,r", [(256, 25), (256, 26), (256, 20), (128, 12), (128, 13), (128, 0),
                                      (128, 3), (64, 10), (64, 70)])
def test_query_dtw(pm, length, r):
    n = 8000 if length == 256 else 6000
    raw = synth.randomwalk(n, length, seed=21)
    qn, _, _ = synth.noisy_queries(6, n, length, data_seed=21)
    qs = np.concatenate([qn, synth.random_queries(3, length)])
    idx, _ = _build(pm, raw, leaf_size=200)
    for k in (1, 4):
        oids, od2 = oracle.knn(raw, qs, k, distance=oracle.DTW, r=r)
        ids, d = _query(pm, idx, qs, k, distance=1, window=r)
        _check_answers(ids, d, oids, od2)
    idx.free()


def test_edge_cases(pm):
    # n = 1, k larger than n: padding with -1 / +inf
    raw = synth.randomwalk(1, 64, seed=3)
    idx, _ = _build(pm, raw, leaf_size=10)
    ids, d = _query(pm, idx, synth.random_queries(2, 64), 4)
    assert np.all(ids[:, 0] == 0) and np.all(ids[:, 1:] == -1) and np.all(np.isinf(d[:, 1:]))
    idx.free()
    # n < k, several series
    raw = synth.randomwalk(5, 64, seed=4)
    idx, _ = _build(pm, raw, leaf_size=2)
    qs = synth.random_queries(3, 64)
    oids, od2 = oracle.knn(raw, qs, 8)
    ids, d = _query(pm, idx, qs, 8)
    _check_answers(ids, d, oids, od2)
    # nq = 0 is a no-op
    e = torch.empty((0, 64), dtype=torch.float32, device="cuda")
    o1, o2 = pm.messi_query(idx, e, 3)
    assert o1.shape == (0, 3)
    idx.free()


def test_many_exact_ties(pm):
    """More equal-distance series than one FP64 recheck pass holds: 3000
    copies of one series (an over-full leaf sorted outside LDS too)."""
    base = synth.randomwalk(2000, 128, seed=5)
    raw = np.concatenate([base, np.repeat(base[7:8], 3000, axis=0)])
    idx, _ = _build(pm, raw, leaf_size=100)
    qs = raw[[7, 11]]
    for k in (1, 3):
        oids, od2 = oracle.knn(raw, qs, k)
        ids, d = _query(pm, idx, qs, k)
        _check_answers(ids, d, oids, od2)
    oids, od2 = oracle.knn(raw, qs[:1], 1)
    ids, d = _query(pm, idx, qs[:1], 1, distance=1, window=5)
    assert ids[0, 0] == 7 and d[0, 0] == 0.0
    idx.free()


def test_query_argument_errors(pm):
    raw = synth.randomwalk(100, 64)
    idx, _ = _build(pm, raw, leaf_size=10)
    q = torch.from_numpy(synth.random_queries(1, 64)).cuda()
    with pytest.raises(pm.MessiError):
        pm.messi_query(idx, q, 0)
    with pytest.raises(pm.MessiError):
        pm.messi_query(idx, q, 2000)
    with pytest.raises(pm.MessiError):
        pm.messi_query(idx, q, 1, distance=5)
    with pytest.raises(pm.MessiError):
        pm.messi_query(idx, q, 1, distance=1, window=-1)
    idx.free()


def test_repeatable(pm):
    raw = synth.randomwalk(20_000, 256, seed=8)
    qs = synth.noisy_queries(12, 20_000, 256, data_seed=8)[0]
    idx, _ = _build(pm, raw)
    first = _query(pm, idx, qs, 5)
    for _ in range(3):
        again = _query(pm, idx, qs, 5)
        assert np.array_equal(first[0], again[0]) and np.array_equal(first[1], again[1])
    idx.free()
