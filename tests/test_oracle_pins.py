"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, a library routine (scipy), a brute force over all warping paths, a
hand-worked case, or an invariant the paper proves (Property 1, Theorem 1,
Theorem 2, Observation 1).
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.special as sp
from scipy.spatial.distance import cdist

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U32 = 2.0 ** -24


# --------------------------------------------------------------- z-norm ---
@pytest.mark.parametrize("n,a,b", [(256, 3.0, 0.5), (128, -7.0, -2.0), (64, 0.0, 1.0), (255, 1e3, 3.0)])
def test_znorm_linear_closed_form(n, a, b):
    """x_t = a + b t has z_t = sgn(b) (t - (n-1)/2) / sqrt((n^2 - 1) / 12)."""
    t = np.arange(n, dtype=np.float64)
    x = (a + b * t).astype(np.float32)
    z = oracle.znorm(x)
    expect = np.sign(b) * (t - (n - 1) / 2.0) / math.sqrt((n * n - 1) / 12.0)
    assert np.max(np.abs(z - expect)) < 2e-5 * max(1.0, abs(a) / max(abs(b), 1e-9) / n)


def test_znorm_constant_is_zero():
    for c in [0.0, 1.5, -3e4]:
        assert np.all(oracle.znorm(np.full(256, c, np.float32)) == 0.0)


def test_znorm_moments_random_walks():
    """Mean 0 and std 1 up to the FP32 rounding of the mean: a sequential
    FP32 sum of len terms is off by at most len u max|x|, i.e. the mean by
    u max|x|, which shifts z by that over sigma."""
    raw = synth.randomwalk(200, 256)
    z = oracle.znorm(raw).astype(np.float64)
    r64 = raw.astype(np.float64)
    tol = 2 * 256 * U32 * np.abs(r64).max(axis=1) / r64.std(axis=1) + 1e-6
    assert np.all(np.abs(z.mean(axis=1)) <= tol)
    assert np.max(np.abs(z.std(axis=1) - 1.0)) < 1e-5


def test_znorm_shift_scale_invariance():
    """z-normalisation removes offset and positive scale (Section 2.1)."""
    raw = synth.randomwalk(20, 256).astype(np.float64)
    for i in range(20):
        z1 = oracle.znorm(raw[i].astype(np.float32))
        z2 = oracle.znorm((4.0 * raw[i] - 9.0).astype(np.float32))
        assert np.max(np.abs(z1 - z2)) < 1e-5


# ------------------------------------------------------------------ PAA ---
def test_paa_constant():
    for c in [0.0, 0.75, -2.5, 12.0]:
        assert np.all(oracle.paa(np.full(256, c, np.float32), 16) == np.float32(c))


def test_paa_integer_inputs_exact():
    """Integer inputs sum exactly in FP32, so each mean is the rounded exact
    fraction."""
    rng = np.random.default_rng(11)
    for w, n in [(16, 256), (16, 128), (8, 64), (4, 100)]:
        x = rng.integers(-1000, 1000, size=n).astype(np.float32)
        p = oracle.paa(x, w)
        m = n // w
        for s in range(w):
            exact = Fraction(int(x[s * m:(s + 1) * m].astype(np.int64).sum()), m)
            assert p[s] == np.float32(float(exact))


def test_paa_linear_closed_form():
    n, w = 256, 16
    m = n // w
    t = np.arange(n, dtype=np.float64)
    z = oracle.znorm((2.0 + 0.25 * t).astype(np.float32))
    p = oracle.paa(z, w)
    s = np.arange(w)
    expect = (s * m + (m - 1) / 2.0 - (n - 1) / 2.0) / math.sqrt((n * n - 1) / 12.0)
    assert np.max(np.abs(p - expect)) < 1e-5


# ----------------------------------------------------------- breakpoints ---
def test_breakpoints_match_normal_quantiles():
    """beta_k = Phi^-1(k/256) rounded to FP32 (scipy's ndtri as reference)."""
    beta = oracle.breakpoints(8)
    ref = sp.ndtri(np.arange(1, 256) / 256.0)
    assert np.array_equal(beta, ref.astype(np.float32))
    assert np.all(np.abs(sp.ndtr(beta.astype(np.float64)) - np.arange(1, 256) / 256.0) < 1e-7)


def test_breakpoints_symmetry_and_nesting():
    beta = oracle.breakpoints(8)
    assert beta[127] == 0.0
    for k in range(1, 256):
        assert beta[256 - k - 1] == -beta[k - 1]
    assert np.all(np.diff(beta) > 0)
    for c in range(1, 8):
        bc = oracle.breakpoints(c)
        step = 1 << (8 - c)
        assert np.array_equal(bc, beta[step - 1::step])


# --------------------------------------------------------------- symbols ---
def test_symbol_hand_cases():
    beta = oracle.breakpoints(8)
    assert oracle.symbol(0.0, beta) == 128  # left-closed: beta_128 = 0 counts
    assert oracle.symbol(-0.0, beta) == 128
    assert oracle.symbol(10.0, beta) == 255
    assert oracle.symbol(-10.0, beta) == 0
    for k in [1, 2, 77, 128, 200, 255]:
        b = float(beta[k - 1])
        assert oracle.symbol(b, beta) == k
        assert oracle.symbol(float(np.nextafter(np.float32(b), np.float32(-np.inf))), beta) == k - 1


def test_symbol_is_normal_cdf_bucket():
    """Away from breakpoints, the symbol is floor(256 Phi(p))."""
    beta = oracle.breakpoints(8)
    rng = np.random.default_rng(5)
    for p in rng.normal(size=3000).astype(np.float32):
        u = sp.ndtr(float(p)) * 256.0
        if abs(u - round(u)) < 1e-4:
            continue
        assert oracle.symbol(float(p), beta) == int(math.floor(u))


def test_words_symbols_bracket_paa():
    """Each symbol is the region holding its segment's PAA (Section 2.2)."""
    raw = synth.randomwalk(300, 256, seed=9)
    W = oracle.words(raw)
    beta = np.concatenate([[-np.inf], oracle.breakpoints(8).astype(np.float64), [np.inf]])
    for i in range(300):
        p = oracle.paa(oracle.znorm(raw[i]), 16).astype(np.float64)
        assert np.all(beta[W[i]] <= p) and np.all(p < beta[W[i].astype(int) + 1])
    Wc = oracle.words(raw, card_bits=4)
    assert np.array_equal(Wc, W >> 4)


# --------------------------------------------------------------- mindist ---
def _random_prefix(word, rng, card_bits=8):
    bits = rng.integers(1, card_bits + 1, size=word.shape[0]).astype(np.uint8)
    sym = (word >> (card_bits - bits)).astype(np.uint8)
    return sym, bits


def test_mindist_lower_bounds_ed_property1():
    """Property 1: node mindist <= ED of every series below the node."""
    rng = np.random.default_rng(3)
    raw = synth.randomwalk(60, 256, seed=21)
    qs = synth.randomwalk(30, 256, seed=22)
    W = oracle.words(raw)
    beta = oracle.breakpoints(8)
    z = oracle.znorm(raw)
    worst = -np.inf
    for j in range(qs.shape[0]):
        zq = oracle.znorm(qs[j])
        qp = oracle.paa(zq, 16)
        for i in range(raw.shape[0]):
            ed2 = oracle.ed2(zq, z[i])
            for _ in range(3):
                sym, bits = _random_prefix(W[i], rng)
                lb2 = oracle.mindist2_ed(qp, sym, bits, beta, 256)
                worst = max(worst, math.sqrt(lb2) - math.sqrt(ed2))
            lb_full = oracle.mindist2_ed(qp, W[i], np.full(16, 8, np.uint8), beta, 256)
            assert lb_full <= ed2 * (1 + 1e-9) + 1e-9
    assert worst <= 1e-6


def test_mindist_of_own_word_is_zero():
    raw = synth.randomwalk(50, 256, seed=4)
    W = oracle.words(raw)
    beta = oracle.breakpoints(8)
    for i in range(50):
        qp = oracle.paa(oracle.znorm(raw[i]), 16)
        assert oracle.mindist2_ed(qp, W[i], np.full(16, 8, np.uint8), beta, 256) == 0.0
        assert oracle.mindist2_ed(qp, W[i] >> 7, np.ones(16, np.uint8), beta, 256) == 0.0


def test_mindist_hand_case():
    """One segment above its box, one below, rest inside: exact value."""
    beta = oracle.breakpoints(8)
    w, n = 16, 256
    sym = np.full(w, 128, np.uint8)
    bits = np.full(w, 8, np.uint8)
    qp = np.array([(beta[127] + beta[128]) / 2] * w, np.float32)  # inside symbol 128
    qp[0] = np.float32(beta[127] - 0.5)  # below box [beta_128, beta_129)
    qp[1] = np.float32(beta[128] + 0.25)  # above the box
    lb2 = oracle.mindist2_ed(qp, sym, bits, beta, n)
    exp = (n / w) * ((float(beta[127]) - float(qp[0])) ** 2 + (float(qp[1]) - float(beta[128])) ** 2)
    assert lb2 == pytest.approx(exp, rel=1e-12)


def test_mindist_dtw_hand_case():
    """The envelope form of the node bound (Section 3.4) on 1-bit boxes,
    whose edges are -inf, beta_128 = 0 and +inf, so every term is exact:
    segment 0's box [0, inf) lies above the upper envelope mean -0.5 (gap
    0.5); segment 1's box (-inf, 0) lies below the lower envelope mean 0.75
    (gap 0.75); segments 2 and 3 overlap their envelope; the rest sit inside
    (-inf, 0).  LB^2 = (256 / 16) (0.5^2 + 0.75^2) = 13."""
    beta = oracle.breakpoints(8)
    assert beta[127] == 0.0
    sym = np.zeros(16, np.uint8)
    sym[[0, 2]] = 1
    bits = np.ones(16, np.uint8)
    up = np.full(16, -1.0, np.float32)
    lp = np.full(16, -1.0, np.float32)
    up[:4] = [-0.5, 1.5, 1.0, 0.5]
    lp[:4] = [-1.0, 0.75, -1.0, -0.25]
    assert oracle.mindist2_dtw(up, lp, sym, bits, beta, 256) == 13.0
    # a swapped envelope would measure segment 0 from -1.0 and segment 1
    # from 1.5 (16 (1 + 2.25) = 52): the roles of U and L are pinned
    assert oracle.mindist2_dtw(lp, up, sym, bits, beta, 256) != 13.0
    # with U = L = the query PAA it is the ED form
    rng = np.random.default_rng(5)
    for _ in range(50):
        qp = rng.standard_normal(16).astype(np.float32)
        s8 = rng.integers(0, 256, 16).astype(np.uint8)
        b8 = rng.integers(1, 9, 16).astype(np.uint8)
        s8 = (s8 >> (8 - b8)).astype(np.uint8)
        assert oracle.mindist2_dtw(qp, qp, s8, b8, beta, 256) == oracle.mindist2_ed(qp, s8, b8, beta, 256)


# ------------------------------------------------------------------- DTW ---
def _golden_dtw():
    rows = []
    with open(os.path.join(GOLDEN, "dtw_hand_cases.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            q, c, r, d, lbk, ed = [s.strip() for s in line.split("|")]
            rows.append((np.array(q.split(), np.float32), np.array(c.split(), np.float32), int(r),
                         float(d), float(lbk), float(ed)))
    return rows


def test_dtw_hand_cases():
    rows = _golden_dtw()
    assert len(rows) >= 5
    for q, c, r, d, lbk, ed in rows:
        assert oracle.dtw2(q, c, r) == d
        U, L = oracle.envelope(q, r)
        assert oracle.lb_keogh2(U, L, c) == lbk
        assert oracle.ed2(q, c) == ed


def _dtw_all_paths(q, c, r):
    """Minimum over every monotone warping path in the band (brute force)."""
    n = len(q)
    best = math.inf
    # a path is a sequence of steps (1,0), (0,1), (1,1) from (0,0) to (n-1,n-1)
    def rec(i, j, acc):
        nonlocal best
        if abs(i - j) > r:
            return
        acc = acc + (float(q[i]) - float(c[j])) ** 2
        if acc >= best:
            return
        if i == n - 1 and j == n - 1:
            best = acc
            return
        if i + 1 < n and j + 1 < n:
            rec(i + 1, j + 1, acc)
        if i + 1 < n:
            rec(i + 1, j, acc)
        if j + 1 < n:
            rec(i, j + 1, acc)

    rec(0, 0, 0.0)
    return best


def test_dtw_equals_min_over_warping_paths():
    rng = np.random.default_rng(8)
    for n in [1, 2, 3, 5, 7]:
        for r in range(0, n + 1):
            for _ in range(4):
                q = rng.normal(size=n).astype(np.float32)
                c = rng.normal(size=n).astype(np.float32)
                assert oracle.dtw2(q, c, r) == pytest.approx(_dtw_all_paths(q, c, r), rel=1e-12)


def test_dtw_window_zero_is_ed_bitwise():
    raw = synth.randomwalk(30, 256, seed=31)
    z = oracle.znorm(raw)
    for i in range(29):
        assert oracle.dtw2(z[i], z[i + 1], 0) == oracle.ed2(z[i], z[i + 1])


def test_lower_bound_chain_and_monotone_in_window():
    """LB_iSAX-DTW <= LB_Keogh <= DTW <= ED, DTW non-increasing in r
    (Section 3.4: LB_Keogh lower-bounds DTW; the envelope PAA bound is the
    segment-mean form of LB_Keogh)."""
    raw = synth.randomwalk(40, 128, seed=41)
    W = oracle.words(raw)
    z = oracle.znorm(raw)
    beta = oracle.breakpoints(8)
    full = np.full(16, 8, np.uint8)
    for j in range(0, 40, 4):
        q = z[j]
        for r in [0, 3, 6, 12, 25]:
            U, L = oracle.envelope(q, r)
            up, lp = oracle.paa(U, 16), oracle.paa(L, 16)
            for i in range(40):
                if i == j:
                    continue
                d = oracle.dtw2(q, z[i], r)
                lbk = oracle.lb_keogh2(U, L, z[i])
                lbi = oracle.mindist2_dtw(up, lp, W[i], full, beta, 128)
                assert math.sqrt(lbi) <= math.sqrt(lbk) + 1e-5
                assert lbk <= d * (1 + 1e-12)
                assert d <= oracle.ed2(q, z[i]) * (1 + 1e-12)
        ds = [oracle.dtw2(q, z[(j + 1) % 40], r) for r in range(0, 128, 7)]
        assert all(a >= b for a, b in zip(ds, ds[1:]))


def test_envelope_brackets_query():
    q = oracle.znorm(synth.randomwalk(1, 256, seed=2)[0])
    for r in [0, 1, 12, 25, 255]:
        U, L = oracle.envelope(q, r)
        assert np.all(U >= q) and np.all(L <= q)
        if r == 0:
            assert np.array_equal(U, q) and np.array_equal(L, q)
        for i in [0, 100, 255]:
            lo, hi = max(0, i - r), min(255, i + r)
            assert U[i] == q[lo:hi + 1].max() and L[i] == q[lo:hi + 1].min()


# ---------------------------------------------------------- brute force ---
def test_knn_ed_matches_scipy_cdist():
    raw = synth.randomwalk(3000, 256, seed=51)
    qs = synth.randomwalk(12, 256, seed=52)
    ids, d2 = oracle.knn(raw, qs, 7)
    z = oracle.znorm(raw).astype(np.float64)
    zq = oracle.znorm(qs).astype(np.float64)
    D = cdist(zq, z, "sqeuclidean")
    for j in range(12):
        order = np.lexsort((np.arange(3000), D[j]))[:7]
        assert np.array_equal(ids[j], order)
        assert np.allclose(d2[j], D[j][order], rtol=1e-12)


def test_knn_ties_break_to_lowest_id_and_chunking():
    raw = synth.randomwalk(500, 64, seed=61)
    raw = np.concatenate([raw, raw[:100], raw[:50]])  # duplicates at 500.. and 600..
    qs = raw[[3, 10, 520]].copy()
    ids, d2 = oracle.knn(raw, qs, 3)
    assert list(ids[0]) == [3, 503, 603]
    assert list(ids[1]) == [10, 510, 610]
    assert list(ids[2]) == [20, 520, 620]
    assert np.all(d2 == 0.0)
    st = oracle.KnnState(qs, 3)
    for a in range(0, raw.shape[0], 97):
        st.scan(raw[a:a + 97], a)
    assert np.array_equal(st.ids, ids) and np.array_equal(st.d2, d2)


def test_knn_dtw_matches_pairwise():
    raw = synth.randomwalk(200, 32, seed=71)
    qs = synth.randomwalk(3, 32, seed=72)
    ids, d2 = oracle.knn(raw, qs, 4, distance=oracle.DTW, r=3)
    z = oracle.znorm(raw)
    for j in range(3):
        zq = oracle.znorm(qs[j])
        D = np.array([oracle.dtw2(zq, z[i], 3) for i in range(200)])
        order = np.lexsort((np.arange(200), D))[:4]
        assert np.array_equal(ids[j], order)


# -------------------------------------------------------- leaf partition ---
def _check_partition(W, perm, leaves, leaf_size, card_bits=8):
    n, w = W.shape
    assert sorted(perm.tolist()) == list(range(n))  # Theorem 1: each series once
    assert leaves["begin"][0] == 0 and leaves["end"][-1] == n
    assert np.all(leaves["begin"][1:] == leaves["end"][:-1])
    prev_key = None
    for L in leaves:
        members = perm[L["begin"]:L["end"]]
        assert len(members) > 0
        assert np.all(np.diff(members) > 0)  # stable: ascending id inside a leaf
        bits = L["bits"][:w].astype(np.int64)
        sym = L["sym"][:w].astype(np.int64)
        assert np.all(bits >= 1) and np.all(bits <= card_bits)
        pref = W[members].astype(np.int64) >> (card_bits - bits)
        assert np.all(pref == sym)  # every member lies in the leaf's box
        if len(members) > leaf_size:
            assert np.all(bits == card_bits)  # over-full only if unsplittable
        key = tuple((sym >> (bits - 1)).tolist())  # root key: first bit of each segment
        if prev_key is not None:
            assert key >= prev_key
        prev_key = key


@pytest.mark.parametrize("n,leaf", [(1, 5), (50, 10), (5000, 100), (20000, 2000), (20000, 37)])
def test_leaf_partition_invariants(n, leaf):
    W = oracle.words(synth.randomwalk(n, 256, seed=81))
    perm, leaves = oracle.leaf_partition(W, leaf)
    _check_partition(W, perm, leaves, leaf)


def test_leaf_partition_boxes_disjoint():
    W = oracle.words(synth.randomwalk(4000, 128, seed=82))
    perm, leaves = oracle.leaf_partition(W, 50)
    # two leaves overlap iff in every segment one prefix extends the other
    for a, b in itertools.combinations(range(min(len(leaves), 300)), 2):
        A, B = leaves[a], leaves[b]
        overlap = True
        for s in range(16):
            ba, bb = int(A["bits"][s]), int(B["bits"][s])
            m = min(ba, bb)
            if (int(A["sym"][s]) >> (ba - m)) != (int(B["sym"][s]) >> (bb - m)):
                overlap = False
                break
        assert not overlap


def test_leaf_partition_duplicates_overfull():
    W = oracle.words(synth.randomwalk(30, 64, seed=83))
    W = np.concatenate([W, np.repeat(W[:1], 40, axis=0)])
    perm, leaves = oracle.leaf_partition(W, 8)
    _check_partition(W, perm, leaves, 8)
    sizes = leaves["end"] - leaves["begin"]
    assert sizes.max() >= 41


def test_leaf_partition_independent_of_input_order():
    W = oracle.words(synth.randomwalk(3000, 256, seed=84))
    perm, leaves = oracle.leaf_partition(W, 60)
    rng = np.random.default_rng(1)
    shuf = rng.permutation(3000)
    perm2, leaves2 = oracle.leaf_partition(W[shuf], 60)
    boxes = lambda Ls: sorted((tuple(L["sym"]), tuple(L["bits"]), int(L["end"] - L["begin"])) for L in Ls)
    assert boxes(leaves) == boxes(leaves2)


def _hand_words(cols, n):
    """n words whose symbols are 0 except the given segment columns."""
    W = np.zeros((n, 16), np.uint8)
    for sg, col in cols.items():
        W[:, sg] = col
    return W


def _leaf_boxes(leaves):
    return [(int(L["begin"]), int(L["end"]), L["sym"][:16].tolist(), L["bits"][:16].tolist())
            for L in leaves]


def _box(changes):
    sym, bits = [0] * 16, [1] * 16
    for sg, (sv, bv) in changes.items():
        sym[sg], bits[sg] = sv, bv
    return sym, bits


def test_leaf_split_most_balanced_segment_hand_case():
    """Section 2.2: a node over the leaf size splits on the segment whose
    next bit divides it most evenly.  Five words under one root key (first
    bit 0 in every segment), leaf size 4.  Second bits (symbol value 64):
    segment 0 has 1s at ids 0 and 2 (|2*2 - 5| = 1), segment 1 at id 1
    (|2 - 5| = 3), the others none (|0 - 5| = 5).  Segment 0 wins; its
    0-child holds ids 1, 3, 4 and its 1-child ids 0, 2, both leaves."""
    W = _hand_words({0: [64, 0, 64, 0, 0], 1: [0, 64, 0, 0, 0]}, 5)
    perm, leaves = oracle.leaf_partition(W, 4)
    assert perm.tolist() == [1, 3, 4, 0, 2]
    assert _leaf_boxes(leaves) == [(0, 3, *_box({0: (0b00, 2)})), (3, 5, *_box({0: (0b01, 2)}))]


def test_leaf_split_ties_to_lowest_segment_hand_case():
    """Segments 2 and 5 both split the five words 2 / 3 (|4 - 5| = 1),
    segment 0 splits them 1 / 4: the tie goes to segment 2, the lower one."""
    W = _hand_words({0: [64, 0, 0, 0, 0], 2: [64, 64, 0, 0, 0], 5: [0, 0, 64, 64, 0]}, 5)
    perm, leaves = oracle.leaf_partition(W, 4)
    assert perm.tolist() == [2, 3, 4, 0, 1]
    assert _leaf_boxes(leaves) == [(0, 3, *_box({2: (0b00, 2)})), (3, 5, *_box({2: (0b01, 2)}))]


def test_leaf_split_two_levels_hand_case():
    """Six words, leaf size 2.  Level 1: segment 1's second bit (64) splits
    ids {0, 2, 4} from {1, 3, 5} evenly (gap 0), beating segment 0 (ids 0, 1:
    gap 2).  Level 2, node {1, 3, 5}: segment 0's second bit (id 1) and
    segment 1's third bit (32; ids 3, 5) both give gap 1: segment 0, the
    lower, splits it into {3, 5} and {1}.  Node {0, 2, 4}: segment 0 (id 0)
    and segment 1's third bit (ids 0, 4) tie again: {2, 4} and {0}."""
    W = _hand_words({0: [64, 64, 0, 0, 0, 0], 1: [96, 0, 64, 32, 96, 32]}, 6)
    perm, leaves = oracle.leaf_partition(W, 2)
    assert perm.tolist() == [3, 5, 1, 2, 4, 0]
    assert _leaf_boxes(leaves) == [
        (0, 2, *_box({0: (0b00, 2), 1: (0b00, 2)})),
        (2, 3, *_box({0: (0b01, 2), 1: (0b00, 2)})),
        (3, 5, *_box({0: (0b00, 2), 1: (0b01, 2)})),
        (5, 6, *_box({0: (0b01, 2), 1: (0b01, 2)})),
    ]


# ------------------------------------------------- index search (Thm 2) ---
@pytest.mark.parametrize("distance,r", [(oracle.ED, 0), (oracle.DTW, 6), (oracle.DTW, 25)])
@pytest.mark.parametrize("k", [1, 5])
def test_index_search_equals_brute_force(distance, r, k):
    n, length = 3000, 128
    raw = synth.randomwalk(n, length, seed=91)
    raw = np.concatenate([raw, raw[:20]])  # exact duplicates force ties
    W = oracle.words(raw)
    perm, leaves = oracle.leaf_partition(W, 100)
    qs = np.concatenate([synth.randomwalk(3, length, seed=92), raw[[5, 17]]])
    bids, bd2 = oracle.knn(raw, qs, k, distance=distance, r=r)
    for j in range(qs.shape[0]):
        ids, d2, st = oracle.index_search(raw, W, perm, leaves, qs[j], k, distance=distance, r=r)
        assert np.array_equal(ids, bids[j])
        assert np.array_equal(d2, bd2[j])
        assert st["bsf_monotone"] == 1  # Observation 1
        assert st["real_dist"] <= raw.shape[0]


def test_index_search_prunes():
    raw = synth.randomwalk(20000, 256, seed=1)
    W = oracle.words(raw)
    perm, leaves = oracle.leaf_partition(W, 2000)
    q = synth.random_queries(4)
    for j in range(4):
        ids, d2, st = oracle.index_search(raw, W, perm, leaves, q[j], 1)
        assert st["real_dist"] < 0.1 * raw.shape[0]


def test_lb_keogh_filtered_scan_equals_plain_scan():
    """Skipping pairs by LB_Keogh <= DTW (Section 3.4) changes no list: same
    ids and bitwise the same FP64 distances as the unfiltered scan, over
    chunks, with exact duplicates (ties) and noisy and random queries."""
    x = synth.randomwalk(6000, 96, seed=1)
    x = np.concatenate([x, x[:40]])
    q = np.concatenate([synth.noisy_queries(6, 6000, 96, data_seed=1)[0],
                        synth.random_queries(2, 96)])
    for r in (0, 4, 20):
        for k in (1, 5):
            a = oracle.KnnState(q, k, oracle.DTW, r)
            b = oracle.KnnState(q, k, oracle.DTW, r, lb_keogh=True)
            for c in range(0, len(x), 1700):
                a.scan(x[c:c + 1700], c)
                b.scan(x[c:c + 1700], c)
            assert np.array_equal(a.ids, b.ids) and np.array_equal(a.d2, b.d2)


def test_lb_improved_hand_case():
    """Worked by hand: q = (0, 3, 0, 0), r = 1 gives U = (3, 3, 3, 0),
    L = (0, 0, 0, 0).  For x = (1, 1, 1, 1), LB_Keogh = 1 (only x_3 leaves
    the envelope); x clamped into it is h = (1, 1, 1, 0), whose envelope is
    U' = (1, 1, 1, 1), L' = (1, 1, 0, 0), and q leaves that by 1 at t = 0 and
    by 2 at t = 1, so LB_Improved = 1 + 1 + 4 = 6.  Every warping path
    visits each q_t, so DTW = 1 + 4 + 1 + 1 = 7 (the diagonal)."""
    q = np.array([0, 3, 0, 0], dtype=np.float32)
    x = np.ones(4, dtype=np.float32)
    U, L = oracle.envelope(q, 1)
    assert list(U) == [3, 3, 3, 0] and list(L) == [0, 0, 0, 0]
    assert oracle.lb_keogh2(U, L, x) == 1.0
    assert oracle.lb_improved2(q, U, L, x, 1) == 6.0
    assert oracle.dtw2(q, x, 1) == 7.0


def test_lb_improved_between_lb_keogh_and_dtw():
    """LB_Keogh <= LB_Improved <= DTW (Lemire 2009, the alternative bound
    of Section 3.4) over random pairs and windows; with r = 0 both bounds
    and DTW coincide with ED."""
    z = oracle.znorm(synth.randomwalk(30, 64, seed=43))
    tighter = 0
    for j in range(0, 30, 3):
        for r in (0, 2, 6, 16):
            U, L = oracle.envelope(z[j], r)
            for i in range(30):
                lbk = oracle.lb_keogh2(U, L, z[i])
                lbi = oracle.lb_improved2(z[j], U, L, z[i], r)
                d = oracle.dtw2(z[j], z[i], r)
                assert lbk <= lbi * (1 + 1e-12) and lbi <= d * (1 + 1e-12)
                tighter += lbi > lbk * (1 + 1e-9)
                if r == 0:
                    assert abs(lbi - oracle.ed2(z[j], z[i])) <= 1e-9 * max(1.0, lbi)
    assert tighter > 100  # the second pass adds something on most pairs


def test_lb_improved_filtered_scan_equals_plain_scan():
    x = synth.randomwalk(4000, 64, seed=2)
    x = np.concatenate([x, x[:30]])
    q = np.concatenate([synth.noisy_queries(5, 4000, 64, data_seed=2)[0],
                        synth.random_queries(2, 64)])
    for r in (3, 12):
        for k in (1, 4):
            a = oracle.KnnState(q, k, oracle.DTW, r)
            b = oracle.KnnState(q, k, oracle.DTW, r, lb_improved=True)
            for c in range(0, len(x), 1500):
                a.scan(x[c:c + 1500], c)
                b.scan(x[c:c + 1500], c)
            assert np.array_equal(a.ids, b.ids) and np.array_equal(a.d2, b.d2)


def test_knn_vote_hand_cases():
    """Majority class of the k nearest neighbours (Section 5.4), worked by
    hand: plain majority, a two-way tie going to the class met first,
    a three-way count tie, k = 1, and lists shorter than k (id -1)."""
    labels = np.array([0, 1, 2, 1, 0, 2, 2, 1, 0, 1], dtype=np.int32)
    ids = np.array([
        [5, 3, 9, -1, -1],   # classes 2, 1, 1 -> 1 (two votes)
        [3, 6, -1, -1, -1],  # 1, 2 tie -> 1 (met first)
        [6, 3, 4, 1, 8],     # 2, 1, 0, 1, 0: 1 and 0 tie at two, 1 met first -> 1
        [4, 2, 5, 0, 7],     # 0, 2, 2, 0, 1: 0 and 2 tie, 0 met first -> 0
        [2, -1, -1, -1, -1],  # k effectively 1 -> 2
        [-1, -1, -1, -1, -1],  # empty -> -1
    ], dtype=np.int64)
    assert oracle.knn_vote(ids, labels, 3).tolist() == [1, 1, 1, 0, 2, -1]
    # labels outside [0, n_classes) are not votes
    bad = labels.copy()
    bad[3] = 7
    bad[9] = -1
    assert oracle.knn_vote(ids[:1], bad, 3).tolist() == [2]


def test_knn_vote_properties():
    """k = 1 gives the nearest neighbour's class; a unanimous list gives
    that class; renaming classes renames the vote."""
    rng = np.random.default_rng(3)
    labels = rng.integers(0, 5, 200).astype(np.int32)
    ids = rng.integers(0, 200, (50, 9)).astype(np.int64)
    assert np.array_equal(oracle.knn_vote(ids[:, :1], labels, 5), labels[ids[:, 0]])
    same = np.repeat(ids[:, :1], 9, axis=1)
    assert np.array_equal(oracle.knn_vote(same, labels, 5), labels[ids[:, 0]])
    perm = rng.permutation(5).astype(np.int32)
    assert np.array_equal(perm[oracle.knn_vote(ids, labels, 5)], oracle.knn_vote(ids, perm[labels], 5))
