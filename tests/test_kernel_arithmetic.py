"""Two arithmetic identities the build and query kernels rely on, checked
by simulation on the CPU (no GPU, no library code).

1. Division by a row's standard deviation.  The build divides every point
   of a row by the same sd, so it refines one reciprocal of sd (one Newton
   step) and corrects each quotient with two FMA residual steps, the way the
   hardware's IEEE division does once its operand scaling is an identity.
   Under the kernel's condition (2^-40 <= sd <= 2^40, |mu| >= 2^-60, so
   every numerator is zero or at least 2^-84 and at most 64 sd), the result
   must be the correctly rounded quotient for any reciprocal estimate within
   one ulp, which the simulation draws at random.

2. Leaf bounds from box ends.  The per-query min-tree holds, for a b-bit
   prefix of a segment, the smallest gap of its symbols' boxes; the batch
   kernel instead takes the gap to the union of those boxes from the first
   box's lower and the last box's upper breakpoint.  For FP32 arithmetic in
   the same order both must give the same bits, also with an envelope
   (upper >= lower PAA) as DTW has."""
import math
import random
from fractions import Fraction

import numpy as np

import oracle

F32 = np.float32


def rn(fr):
    """Round a Fraction to the nearest float32 (ties to even), exactly."""
    c = F32(float(fr))  # a neighbour of the true value
    cands = {c, np.nextafter(c, F32(np.inf)), np.nextafter(c, F32(-np.inf))}

    def key(v):
        return (abs(Fraction(float(v)) - fr), int(np.array(v, F32).view(np.uint32)) & 1)

    return F32(min(cands, key=key))


def fma(a, b, c):
    return rn(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def div_by(num, den, r):
    m = rn(Fraction(float(num)) * Fraction(float(r)))
    e1 = fma(-den, m, num)
    q1 = fma(e1, r, m)
    e2 = fma(-den, q1, num)
    return fma(e2, r, q1)


def test_hoisted_reciprocal_division_is_correctly_rounded():
    rnd = random.Random(7)
    for _ in range(2500):
        sd = F32(2.0 ** rnd.uniform(-40, 40) * rnd.uniform(1, 2))
        sd = min(max(sd, F32(2.0 ** -40)), F32(2.0 ** 40))
        r0 = rn(Fraction(1) / Fraction(float(sd)))
        step = rnd.choice([-1, 0, 1])  # a reciprocal estimate within one ulp
        if step:
            r0 = np.nextafter(r0, F32(math.copysign(np.inf, step)))
        e0 = fma(-sd, r0, F32(1.0))
        r = fma(e0, r0, r0)
        if rnd.random() < 0.15:  # small numerators, down to the 2^-84 floor
            num = F32(2.0 ** rnd.uniform(-84, -30)) * F32(rnd.choice([-1, 1]))
        else:
            num = F32(float(sd) * rnd.uniform(-64, 64))
        want = rn(Fraction(float(num)) / Fraction(float(sd)))
        got = div_by(num, sd, r)
        assert got == want, (num, sd, got, want)


def test_a_dropped_correction_is_caught():
    """The check above tells a plain multiply by the refined reciprocal (the
    corrections dropped) from the correctly rounded quotient."""
    rnd = random.Random(3)
    bad = 0
    for _ in range(400):
        sd = F32(2.0 ** rnd.uniform(-10, 10) * rnd.uniform(1, 2))
        r0 = rn(Fraction(1) / Fraction(float(sd)))
        r = fma(fma(-sd, r0, F32(1.0)), r0, r0)
        num = F32(float(sd) * rnd.uniform(-64, 64))
        q = rn(Fraction(float(num)) * Fraction(float(r)))  # no correction
        bad += q != rn(Fraction(float(num)) / Fraction(float(sd)))
    assert bad > 0


def tree_value(bp, pu, pl, b, y, cb, fm):
    """The min-tree's entry for prefix (b, y): the smallest value over the
    prefix's symbols of fm * g^2, g the gap of the envelope to the box."""
    best = None
    width = 1 << (cb - b)
    for j in range(y * width, (y + 1) * width):
        g = np.maximum(F32(bp[j] - pu), F32(0)) + np.maximum(F32(pl - bp[j + 1]), F32(0))
        v = F32(fm * F32(g * g))
        best = v if best is None else min(best, v)
    return best


def union_value(bp, pu, pl, b, y, cb, fm):
    lo, hi = bp[y << (cb - b)], bp[(y + 1) << (cb - b)]
    g = np.maximum(F32(lo - pu), F32(0)) + np.maximum(F32(pl - hi), F32(0))
    return F32(fm * F32(g * g))


def test_leaf_box_gap_equals_the_min_tree_value():
    cb = 8
    bp = np.concatenate([[-np.inf], oracle.breakpoints(cb), [np.inf]]).astype(F32)
    rng = np.random.default_rng(11)
    fm = F32(16.0)
    for _ in range(600):
        c = F32(rng.normal(0, 1.5))
        half = F32(abs(rng.normal(0, 0.3))) if rng.random() < 0.5 else F32(0)
        pu, pl = F32(c + half), F32(c - half)  # DTW envelope, or ED (pu = pl)
        b = int(rng.integers(0, cb + 1))
        y = int(rng.integers(0, 1 << b)) if b else 0
        assert union_value(bp, pu, pl, b, y, cb, fm) == tree_value(bp, pu, pl, b, y, cb, fm)
    # on a breakpoint, and between two boxes of the prefix
    for j in (1, 37, 128, 200, 255):
        for b in range(cb + 1):
            y = j >> (cb - b)
            v = bp[j]
            assert union_value(bp, v, v, b, y, cb, fm) == tree_value(bp, v, v, b, y, cb, fm)


def test_an_off_by_one_box_end_is_caught():
    """The comparison above tells apart a union whose upper end is taken one
    breakpoint too low."""
    cb = 8
    bp = np.concatenate([[-np.inf], oracle.breakpoints(cb), [np.inf]]).astype(F32)
    rng = np.random.default_rng(5)
    fm = F32(16.0)
    diffs = 0
    for _ in range(300):
        p = F32(rng.normal(0, 1.5))
        b = int(rng.integers(1, cb + 1))
        y = int(rng.integers(0, 1 << b))
        lo, hi = bp[y << (cb - b)], bp[((y + 1) << (cb - b)) - 1]
        g = np.maximum(F32(lo - p), F32(0)) + np.maximum(F32(p - hi), F32(0))
        diffs += F32(fm * F32(g * g)) != tree_value(bp, p, p, b, y, cb, fm)
    assert diffs > 0
