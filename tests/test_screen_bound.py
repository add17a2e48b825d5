"""The BF16 screen's dot-product error bound, checked by simulation on the
CPU (no GPU, no library code).

The screen computes s~ = sum_i bf16(q_i) * bf16(x_i) with FP32
accumulation and keeps a pair unless its distance lower bound, built from
s~ and an error term, exceeds the k-th best.  Rounding each operand to BF16
(8 significant bits, round to nearest even, unit u_b = 2^-8) and summing
len exact products in FP32 (unit 2^-23, order not specified) gives

    |s~ - q.x| <= [(2 u_b + u_b^2) + gamma_len (1 + u_b)^2] * |q| |x|,
    gamma_len = len 2^-23 / (1 - len 2^-23),

by the standard product and summation error bounds and Cauchy-Schwarz.
These tests draw z-normalised-like vectors, vectors at BF16 rounding
midpoints (where the operand bound is tight) and aligned pairs (where
Cauchy-Schwarz is tight), accumulate in several orders, and check that
the bound holds and is not loose by more than a modest factor on the
tight cases.  A derivation that counted one operand's rounding only fails
them; the accumulation term (about 0.4% of the bound at 256 points) is
checked only in that the bound holds with it."""
import numpy as np
import pytest

U_B = 2.0 ** -8
U_32 = 2.0 ** -23


def bf16(v):
    """Round float32 values to BF16 (nearest, ties to even), as float32."""
    b = np.ascontiguousarray(v, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def bound(q, x):
    n = q.shape[-1]
    gamma = n * U_32 / (1.0 - n * U_32)
    cq = np.linalg.norm(q.astype(np.float64), axis=-1)
    cx = np.linalg.norm(x.astype(np.float64), axis=-1)
    return ((2 * U_B + U_B * U_B) + gamma * (1 + U_B) ** 2) * cq * cx


def sums(p):
    """FP32 sums of the rows of p (exact products) in several orders."""
    out = []
    acc = np.zeros(p.shape[0], np.float32)
    for i in range(p.shape[1]):  # one after another
        acc = (acc + p[:, i]).astype(np.float32)
    out.append(acc)
    out.append(np.sum(p, axis=1, dtype=np.float32))  # numpy's pairwise order
    acc = np.zeros(p.shape[0], np.float32)
    for i in range(0, p.shape[1], 4):  # blocks of four, then the running sum
        blk = np.zeros(p.shape[0], np.float32)
        for j in range(i, min(i + 4, p.shape[1])):
            blk = (blk + p[:, j]).astype(np.float32)
        acc = (acc + blk).astype(np.float32)
    out.append(acc)
    acc = np.zeros(p.shape[0], np.float32)
    for i in range(p.shape[1] - 1, -1, -1):  # reversed
        acc = (acc + p[:, i]).astype(np.float32)
    out.append(acc)
    return out


def check(q, x):
    exact = np.einsum("ij,ij->i", q.astype(np.float64), x.astype(np.float64))
    qb, xb = bf16(q), bf16(x)
    prods = (qb * xb).astype(np.float32)
    # a product of two BF16 values has at most 16 significant bits: exact in FP32
    assert np.array_equal(prods.astype(np.float64), qb.astype(np.float64) * xb.astype(np.float64))
    bnd = bound(q, x)
    worst = 0.0
    for s in sums(prods):
        err = np.abs(s.astype(np.float64) - exact)
        assert np.all(err <= bnd), (err.max(), bnd[err.argmax()])
        worst = max(worst, float(np.max(err / bnd)))
    return worst


def znorm(v):
    v = v - v.mean(axis=1, keepdims=True)
    return (v / v.std(axis=1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("length", [64, 128, 256, 512])
def test_bound_holds_on_random_walks(length):
    rng = np.random.default_rng(length)
    q = znorm(np.cumsum(rng.standard_normal((200, length)), axis=1))
    x = znorm(np.cumsum(rng.standard_normal((200, length)), axis=1))
    check(q, x)
    check(q, q + np.float32(0.01) * rng.standard_normal(q.shape).astype(np.float32))


@pytest.mark.parametrize("length", [64, 256])
def test_bound_is_tight_at_rounding_midpoints(length):
    # every operand just above a power of two and just below a BF16
    # midpoint rounds down by almost u_b of its value, all products share a
    # sign and q = x: both the operand bound and Cauchy-Schwarz are nearly
    # attained
    rng = np.random.default_rng(7)
    mant = rng.integers(0, 4, size=(50, length))
    e = rng.integers(-3, 3, size=(50, length)).astype(np.float64)
    v = (1.0 + (mant + 0.5 - 2.0 ** -6) / 128.0) * 2.0 ** e  # just under the midpoint
    q = v.astype(np.float32)
    worst = check(q, q.copy())
    assert worst > 0.85, worst  # the bound is within 1/0.85 of the error here


def test_one_operand_term_alone_fails_at_midpoints():
    # the same tight case against a bound that counts one rounding only:
    # the error exceeds it, so the factor 2 u_b is needed
    rng = np.random.default_rng(8)
    mant = rng.integers(0, 128, size=(20, 256))
    q = ((1.0 + (mant + 0.5 - 2.0 ** -6) / 128.0)).astype(np.float32)
    exact = np.einsum("ij,ij->i", q.astype(np.float64), q.astype(np.float64))
    qb = bf16(q)
    s = np.sum((qb * qb).astype(np.float32), axis=1, dtype=np.float32)
    err = np.abs(s.astype(np.float64) - exact)
    one = U_B * np.linalg.norm(q.astype(np.float64), axis=1) ** 2
    assert np.all(err > one)


def test_bf16_rounding_is_nearest_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even 1
    v = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9, -(1.0 + 2.0 ** -8)], np.float32)
    assert bf16(v).tolist() == [1.0, 1.0 + 2.0 ** -6, 1.0, -1.0]


# ----------------------------------------------------------------------------
# The whole folded drop test, simulated in FP32 step by step.
#
# The screen keeps a pair unless
#   x = fma(-2, s~, fma(-a_q, s_x, R_q + C_x)) > 0,
#   R_q = fl(fl(|q|^2) (1 - c_abs)) - thr   (two FP32 roundings),
#   C_x = fl(fl(|x|^2) (1 - c_abs)),  a_q = fl(c_dot sqrt(fl(|q|^2))),
#   s_x = sqrt(fl(|x|^2)),
# with the squared norms summed in FP64 and rounded to FP32 once, and
# c_abs = 2^-17 covering those roundings and the FP32 evaluation.  A drop
# is sound iff it implies |q - x|^2 > thr for the FP32 rows.  The cases
# below stress the c_abs term: zero and tiny rows (no dot-product slack at
# all), identical rows at BF16 rounding midpoints (the dot-product slack
# used up), near copies (large norms, small distance) and rows with a large
# offset (raw indexes), each with the threshold at the smallest FP32 value
# not below the exact distance, where a drop would be wrong.

from fractions import Fraction

C_ABS = 2.0 ** -17


def c_dot(n):
    ub = U_B
    g = n * U_32 / (1.0 - n * U_32)
    return np.float32(np.nextafter(np.float32(2.0 * ((2 * ub + ub * ub) + g * (1 + ub) ** 2)
                                              * (1.0 + 2.0 ** -10)), np.float32(np.inf)))


def rn32(fr):
    """Round a Fraction to the nearest FP32 value (ties to even)."""
    if fr == 0:
        return np.float32(0.0)
    sign = -1 if fr < 0 else 1
    a = abs(fr)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, -126)
    scale = Fraction(2) ** (23 - e)
    m = a * scale
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return np.float32(sign * float(Fraction(fl) / scale))


def fma32(a, b, c):
    return rn32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def ru32(v):
    """Smallest FP32 value not below the float64 v."""
    f = np.float32(v)
    return f if float(f) >= v else np.nextafter(f, np.float32(np.inf))


def folded_drop(q, x, s, thr, one_m=np.float32(1.0 - C_ABS), cd=None):
    """The screen's drop decision for one pair, FP32 step by step."""
    n = q.shape[0]
    cd = c_dot(n) if cd is None else cd
    qn = np.float32(np.sum(q.astype(np.float64) ** 2))
    xn = np.float32(np.sum(x.astype(np.float64) ** 2))
    R = np.float32(np.float32(qn * one_m) - thr)
    a = np.float32(cd * np.sqrt(qn, dtype=np.float32))
    cx = np.float32(xn * one_m)
    sx = np.sqrt(xn, dtype=np.float32)
    inner = fma32(-a, sx, np.float32(R + cx))
    return fma32(np.float32(-2.0), s, inner) > 0


def screen_cases():
    rng = np.random.default_rng(11)
    out = []
    for n in (128, 256):
        zq = znorm(np.cumsum(rng.standard_normal((6, n)), axis=1))
        out += [(zq[i], np.zeros(n, np.float32)) for i in range(3)]  # flat rows
        out += [(zq[i], (1e-4 * rng.standard_normal(n)).astype(np.float32)) for i in range(3)]
        out += [(zq[i], (zq[i] + np.float32(1e-3) * rng.standard_normal(n)).astype(np.float32))
                for i in range(6)]  # near copies
        mant = rng.integers(0, 4, size=(3, n))
        v = ((1.0 + (mant + 0.5 - 2.0 ** -6) / 128.0) * 2.0 ** rng.integers(-2, 2, size=(3, n)))
        out += [(r.astype(np.float32), r.astype(np.float32)) for r in v]  # midpoints, q = x
        off = (100.0 + rng.standard_normal((4, n))).astype(np.float32)
        out += [(off[0], off[1]), (off[2], off[2] + np.float32(0.01)), (off[3], np.zeros(n, np.float32))]
    return out


def test_folded_test_never_drops_a_pair_at_the_threshold():
    for q, x in screen_cases():
        d2 = float(np.sum((q.astype(np.float64) - x.astype(np.float64)) ** 2))
        prods = (bf16(q) * bf16(x)).astype(np.float32)[None, :]
        for s in sums(prods):
            for thr in (ru32(d2), np.nextafter(ru32(d2), np.float32(np.inf)), ru32(d2 * 1.001)):
                assert not folded_drop(q, x, s[0], thr), (d2, float(thr))


def test_folded_test_still_drops_far_pairs():
    # the slack is small: pairs well beyond the threshold are dropped
    rng = np.random.default_rng(12)
    q = znorm(np.cumsum(rng.standard_normal((20, 256)), axis=1))
    x = znorm(np.cumsum(rng.standard_normal((20, 256)), axis=1))
    dropped = 0
    for i in range(20):
        d2 = float(np.sum((q[i].astype(np.float64) - x[i].astype(np.float64)) ** 2))
        s = np.sum((bf16(q[i]) * bf16(x[i])).astype(np.float32), dtype=np.float32)
        dropped += folded_drop(q[i], x[i], s, np.float32(0.9 * d2))
    assert dropped == 20


def test_norm_terms_need_the_lower_factor():
    # scaling the norms up by (1 + c_abs) instead of down drops a flat row
    # exactly at the threshold: the sign of the c_abs term matters
    wrong = 0
    for q, x in screen_cases():
        d2 = float(np.sum((q.astype(np.float64) - x.astype(np.float64)) ** 2))
        s = np.sum((bf16(q) * bf16(x)).astype(np.float32), dtype=np.float32)
        wrong += folded_drop(q, x, s, ru32(d2), one_m=np.float32(1.0 + C_ABS))
    assert wrong > 0


def test_rn32_rounds_like_the_fp32_conversion():
    rng = np.random.default_rng(14)
    v = rng.standard_normal(2000) * 10.0 ** rng.integers(-8, 8, 2000)
    for x in v:
        assert rn32(Fraction(float(x))) == np.float32(x)
    # exact halfway cases go to the even neighbour
    assert rn32(Fraction(1) + Fraction(1, 2 ** 24)) == np.float32(1.0)
    assert rn32(Fraction(1) + Fraction(3, 2 ** 24)) == np.float32(1.0 + 2.0 ** -22)
