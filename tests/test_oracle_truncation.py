"""Pin of the oracle's truncation rule (Section III-B, non-Clifford
paragraph: a merged term whose modulus is strictly below the threshold is
removed).  The ground truth here is exact rational arithmetic:
|c| < t  <=>  re^2 + im^2 < t^2 over the rationals (Python Fractions), so a
rule that squares in floating point (and underflows below t ~ 1e-154,
overflows above ~1e154, or rounds a near-tie the wrong way) fails it."""
import math
import random
from fractions import Fraction

import numpy as np

from oracle import oracle as O


def _exact_below(re, im, t):
    if not t > 0:
        return False
    return Fraction(re) ** 2 + Fraction(im) ** 2 < Fraction(t) ** 2


def _cases():
    rng = random.Random(25974)
    cases = []
    # exact ties |c| = t (3-4-5 triangles scaled by powers of two) and their neighbours
    for e in (-1070, -1000, -600, -300, -160, -80, 0, 40, 300, 600, 1000):
        re, im, t = math.ldexp(3.0, e), math.ldexp(4.0, e), math.ldexp(5.0, e)
        cases += [(re, im, t), (re, im, math.nextafter(t, math.inf)),
                  (re, im, math.nextafter(t, 0.0)), (-re, im, t), (im, -re, t)]
    # zeros, subnormals, a lone component, thresholds where squares underflow
    for t in (1e-300, 5e-324, 1e-320, 1e-200, 1e-160, 1.5e-154, 1e-10, 1.0, 1e160, 1e300):
        cases += [(0.0, 0.0, t), (-0.0, 0.0, t), (5e-324, 0.0, t), (0.0, t, t),
                  (math.nextafter(t, 0.0), 0.0, t), (t / 2, t / 2, t),
                  (t * 0.7071067811865476, t * 0.7071067811865476, t),
                  (t * 0.7071067811865475, t * 0.7071067811865475, t)]
    # near ties drawn at random: im chosen so that re^2 + im^2 is close to t^2
    for _ in range(3000):
        e = rng.choice([-1060, -700, -400, -160, -60, -10, 0, 10, 60, 160, 400, 700, 1000])
        t = math.ldexp(rng.uniform(1.0, 2.0), e)
        re = t * rng.uniform(0.0, 1.0)
        im = math.sqrt(max(t * t - re * re, 0.0)) if abs(e) < 400 else t * math.sqrt(
            max(1.0 - (re / t) ** 2, 0.0))
        for _ in range(rng.randrange(0, 4)):
            im = math.nextafter(im, rng.choice([0.0, math.inf]))
        if rng.random() < 0.5:
            re, im = im, re
        cases.append((re * rng.choice([1, -1]), im * rng.choice([1, -1]), t))
    # a term with one component far below the other
    for _ in range(500):
        t = math.ldexp(1.0, rng.randrange(-1000, 1000))
        cases.append((math.nextafter(t, 0.0), t * math.ldexp(1.0, -rng.randrange(20, 80)), t))
    return cases


def test_truncation_is_exact():
    cases = _cases()
    n = 40  # distinct strings: term u has the X bits of u
    m = 1
    checked = 0
    by_t = {}
    for re, im, t in cases:
        by_t.setdefault(t, []).append((re, im))
    for t, vals in by_t.items():
        m = len(vals)
        x = np.arange(1, m + 1, dtype=np.uint64).reshape(m, 1)
        z = np.zeros((m, 1), np.uint64)
        c = np.array([complex(re, im) for re, im in vals], np.complex128)
        kept = O.merge(O.Sum(n, x, z, None, c), drop_abs=t)
        got = {int(v) for v in kept.x[:, 0]}
        for u, (re, im) in enumerate(vals):
            want_kept = not _exact_below(re, im, t)
            assert ((u + 1) in got) == want_kept, (re, im, t)
            checked += 1
    assert checked == len(cases)


def test_zero_sum_dropped_at_tiny_threshold():
    """A coefficient that cancels to exactly zero lies below any positive
    threshold, 1e-300 included (a squared threshold would underflow to 0 and
    keep it)."""
    x = np.array([[1], [1]], np.uint64)
    z = np.zeros((2, 1), np.uint64)
    S = O.Sum(4, x, z, None, np.array([0.5 + 0.25j, -0.5 - 0.25j]))
    assert O.merge(S, drop_abs=1e-300).x.shape[0] == 0
    assert O.merge(S, drop_abs=0.0).x.shape[0] == 1  # nothing is below 0
    assert O.merge(S, drop_abs=-1.0).x.shape[0] == 1
