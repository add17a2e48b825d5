"""Pins of the oracle's non-normalised mode and of its subsequence windows.

The paper's index also serves series taken as they are, without
z-normalisation (Section 1), and subsequence search by indexing every
sliding window of a long series (Section 2.1).  Each test checks the oracle
against something other than itself: scipy's distances, a dynamic program
written out here, closed forms of the symbols, Theorem 2 (the index search
equals the brute-force answer), or the normalised mode it must reduce to.
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
import synth


def _offset_rows(n, length, seed):
    """Random walks with per-row offsets and scales: raw values far from the
    unit-variance range the breakpoints were made for."""
    x = synth.randomwalk(n, length, seed=seed).astype(np.float64)
    rng = np.random.default_rng(seed)
    x = x * rng.uniform(0.2, 4.0, (n, 1)) + rng.uniform(-300.0, 300.0, (n, 1))
    return x.astype(np.float32)


def test_raw_mode_on_normalised_rows_equals_normalised_mode():
    raw = synth.randomwalk(1500, 128, seed=3)
    qs = synth.randomwalk(6, 128, seed=4)
    z, zq = oracle.znorm(raw), oracle.znorm(qs)
    w_norm = oracle.words(raw)
    ids_n, d2_n = oracle.knn(raw, qs, 5)
    ids_d, d2_d = oracle.knn(raw, qs, 3, distance=oracle.DTW, r=9)
    with oracle.raw_mode():
        assert np.array_equal(oracle.words(z), w_norm)
        ids_r, d2_r = oracle.knn(z, zq, 5)
        ids_rd, d2_rd = oracle.knn(z, zq, 3, distance=oracle.DTW, r=9)
    assert np.array_equal(ids_r, ids_n) and np.array_equal(d2_r, d2_n)
    assert np.array_equal(ids_rd, ids_d) and np.array_equal(d2_rd, d2_d)
    # and the mode switch is scoped: the default is normalised again
    assert np.array_equal(oracle.words(raw), w_norm)


def test_raw_knn_ed_matches_scipy_cdist():
    raw = _offset_rows(2500, 64, seed=7)
    qs = np.concatenate([_offset_rows(5, 64, seed=8), raw[[11, 2000]]])
    with oracle.raw_mode():
        ids, d2 = oracle.knn(raw, qs, 6)
    D = cdist(qs.astype(np.float64), raw.astype(np.float64), "sqeuclidean")
    for j in range(len(qs)):
        order = np.lexsort((np.arange(len(raw)), D[j]))[:6]
        assert np.array_equal(ids[j], order)
        assert np.allclose(d2[j], D[j][order], rtol=1e-12)
    assert ids[5, 0] == 11 and d2[5, 0] == 0.0


def _dtw2_dp(a, b, r):
    """Sakoe-Chiba banded DTW with squared point costs, as a plain dynamic
    program over the (len+1)^2 table."""
    n = len(a)
    D = np.full((n + 1, n + 1), np.inf)
    D[0, 0] = 0.0
    for i in range(1, n + 1):
        for j in range(max(1, i - r), min(n, i + r) + 1):
            c = (float(a[i - 1]) - float(b[j - 1])) ** 2
            D[i, j] = c + min(D[i - 1, j], D[i, j - 1], D[i - 1, j - 1])
    return D[n, n]


def test_raw_knn_dtw_matches_dynamic_program():
    raw = _offset_rows(60, 24, seed=9)
    qs = _offset_rows(3, 24, seed=10)
    with oracle.raw_mode():
        ids, d2 = oracle.knn(raw, qs, 4, distance=oracle.DTW, r=3)
    for j in range(3):
        D = np.array([_dtw2_dp(qs[j], raw[i], 3) for i in range(60)])
        order = np.lexsort((np.arange(60), D))[:4]
        assert np.array_equal(ids[j], order)
        assert np.allclose(d2[j], D[order], rtol=1e-12)


def test_raw_words_saturate_and_bracket_the_paa():
    beta = oracle.breakpoints(8).astype(np.float64)
    hi = np.full((3, 64), 50.0, dtype=np.float32)      # above every breakpoint
    lo = np.full((3, 64), -50.0, dtype=np.float32)     # below every breakpoint
    with oracle.raw_mode():
        assert np.all(oracle.words(hi) == 255) and np.all(oracle.words(lo) == 0)
        x = synth.randomwalk(400, 128, seed=12) * np.float32(0.1)
        W = oracle.words(x)
    paa = x.astype(np.float64).reshape(400, 16, 8).mean(axis=2)
    want = np.searchsorted(beta, paa, side="right")
    gap = np.min(np.abs(paa[..., None] - beta[None, None, :]), axis=2)
    far = gap > 1e-5  # FP32 segment means decide symbols only near a breakpoint
    assert far.mean() > 0.99
    assert np.array_equal(W[far], want[far])


@pytest.mark.parametrize("distance,r", [(oracle.ED, 0), (oracle.DTW, 8)])
def test_raw_index_search_equals_brute_force(distance, r):
    raw = _offset_rows(2000, 64, seed=13)
    raw[:, :] *= np.float32(0.02)  # spread the words over many leaves
    raw = np.concatenate([raw, raw[:10]])
    qs = np.concatenate([_offset_rows(3, 64, seed=14) * np.float32(0.02), raw[[4, 1500]]])
    with oracle.raw_mode():
        W = oracle.words(raw)
        perm, leaves = oracle.leaf_partition(W, 50)
        bids, bd2 = oracle.knn(raw, qs, 3, distance=distance, r=r)
        for j in range(len(qs)):
            ids, d2, st = oracle.index_search(raw, W, perm, leaves, qs[j], 3, distance=distance, r=r)
            assert np.array_equal(ids, bids[j]) and np.array_equal(d2, bd2[j])
            assert st["bsf_monotone"] == 1
    assert len(leaves) > 20


@pytest.mark.parametrize("stride", [1, 3, 8])
def test_windows_are_the_sliding_windows(stride):
    s = synth.randomwalk(1, 1000, seed=15)[0]
    W = oracle.windows(s, 50, stride)
    assert W.shape == ((1000 - 50) // stride + 1, 50)
    for i in [0, 1, len(W) // 2, len(W) - 1]:
        assert np.array_equal(W[i], s[i * stride:i * stride + 50])
    # a window of the series itself is found at distance 0 at its start
    q = s[stride * 17:stride * 17 + 50][None, :]
    with oracle.raw_mode():
        ids, d2 = oracle.knn(W, q, 1)
    assert ids[0, 0] == 17 and d2[0, 0] == 0.0
