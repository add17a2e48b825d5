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
