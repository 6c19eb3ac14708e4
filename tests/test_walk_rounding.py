"""The lane walk's exact-rounding argument, checked on the host in exact
rational arithmetic (the walk itself is checked against the oracle by the GPU
parity tests).  The walk takes each slope bound of the greedy fit (the
interval of fixed-point slopes a key allows, Sec. II-A) as one FMA of the
key's numerator with a correctly rounded 1/d, rounded into the mantissa of
1.5 * 2^52, with no remainder correction:

  floor(y / d) = round((y + 1/2 - d/2) * RN(1/d))   for integers |y| < 2^49,
  ceil(x / d)  = floor((x + d - 1) / d),

and it forms the numerators from a per-key term (K' 2^F +- e/2) and a
per-segment term, in FP64 adds that must be exact.  Python floats are IEEE
doubles and float(Fraction) rounds to nearest even, so one hardware FMA is
float(Fraction(a) * Fraction(b) + Fraction(c))."""
import random
from fractions import Fraction

import pytest

K_ROUND = 6755399441055744.0  # 1.5 * 2^52


def fma(a: float, b: float, c: float) -> float:
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def exact_add(a: float, b: float) -> float:
    r = a + b
    assert Fraction(r) == Fraction(a) + Fraction(b), (a, b)
    return r


def walk_bounds(base: int, D: int, s: int, d: int, eps: int, F: int):
    """The (lower, upper) slope bounds of key e = s + d, anchor s, as the walk
    computes them: per-key terms at e, per-segment terms at the anchor."""
    scf = float(1 << F)
    eps_lo = float(eps) * scf
    eps_hi = (float(eps) + 1.0) * scf - 1.0
    c_lo, c_hi = -eps_lo - 0.5, eps_hi + 0.5
    e = s + d
    x_s = float(base) * scf            # K'(s) 2^F
    x_e = float(base + D) * scf        # K'(e) 2^F
    pk, qk = exact_add(x_e, e / 2), exact_add(x_e, -e / 2)
    ca = exact_add(c_lo, -exact_add(x_s, s / 2))
    cb = exact_add(c_hi, -exact_add(x_s, -s / 2))
    inv = 1.0 / d                      # correctly rounded, like the LDS table
    lo = fma(exact_add(pk, ca), inv, K_ROUND) - K_ROUND
    hi = fma(exact_add(qk, cb), inv, K_ROUND) - K_ROUND
    return lo, hi


def exact_bounds(D: int, d: int, eps: int, F: int):
    num_lo = (D - eps) << F if D >= eps else -((eps - D) << F)
    num_hi = ((D + eps + 1) << F) - 1
    return -((-num_lo) // d), num_hi // d


def test_floor_identity_random():
    rng = random.Random(11)
    for _ in range(20000):
        d = rng.randint(1, 4097)
        y = rng.randint(-(1 << 49) + 1, (1 << 49) - 1)
        if rng.random() < 0.3:  # on and next to multiples of d
            y = (y // d) * d + rng.choice((0, 1, -1, d - 1))
            y = max(-(1 << 49) + 1, min((1 << 49) - 1, y))
        yp = Fraction(y) + Fraction(1, 2) - Fraction(d, 2)
        q = fma(float(yp), 1.0 / d, K_ROUND) - K_ROUND
        assert q == y // d, (y, d, q)


@pytest.mark.parametrize("F", [0, 8, 20])
def test_walk_bounds_match_exact(F):
    rng = random.Random(100 + F)
    lim = 1 << (49 - F)  # the walk's fast path needs (span + eps + 1) 2^F < 2^49
    for _ in range(8000):
        eps = rng.choice((0, 1, 3, 63, 255, 1 << 10, (1 << 20) - 1))
        eps = min(eps, lim // 4)
        span = rng.randint(1, lim - eps - 2)
        D = rng.randint(0, span)
        d = rng.randint(1, 4096)
        s = rng.randint(0, 4096 - d)
        base = rng.randint(0, span - D)
        assert walk_bounds(base, D, s, d, eps, F) == exact_bounds(D, d, eps, F), (base, D, s, d, eps, F)


def test_walk_bounds_extremes():
    # largest spans the fast path admits, smallest and largest distances,
    # numerators on multiples of d, keys below and above eps of the anchor
    for F in (0, 20):
        lim = 1 << (49 - F)
        for eps in (0, 63, 4095):
            span = lim - eps - 2
            for d in (1, 2, 3, 1023, 1024, 1025, 4096):
                for D in (0, 1, eps, eps + 1, span, span - 1, (span // d) * d, eps + d):
                    if D > span:
                        continue
                    for s in (0, 4096 - d):
                        for base in (0, span - D):
                            assert walk_bounds(base, D, s, d, eps, F) == exact_bounds(D, d, eps, F)


def test_planted_mistake_is_caught():
    """Dropping the half-distance offset (rounding y / d to nearest) must fail."""
    bad = 0
    rng = random.Random(5)
    for _ in range(2000):
        d = rng.randint(2, 4097)
        y = rng.randint(0, 1 << 40)
        q = fma(float(y), 1.0 / d, K_ROUND) - K_ROUND
        bad += q != y // d
    assert bad > 0
