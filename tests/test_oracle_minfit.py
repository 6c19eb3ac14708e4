"""Pins of the oracle's fewest-segment fit (``fit="min"``), against brute
force that shares nothing with the oracle's cone arithmetic:

* a segment [s, e) of the anchored class is feasible when some integer slope
  A keeps every key within eps of K[s] + floor(A (i - s) / 2^F) (Def. 2,
  Eq. 1 with anchored fixed-point segments); the brute force tries every A
  in a range that provably holds all feasible ones;
* the minimum number of segments is a shortest path over all feasible
  segments (dynamic programming over every segmentation);
* of the minimum segmentations the oracle must return the one whose every
  boundary lies earliest (the componentwise minimum of the boundary
  vectors, which the brute force finds by enumerating all of them);
* each stored slope is floor((lo + hi) / 2) of that segment's full integer
  interval [lo, hi] of feasible slopes (negative ones included), clamped to
  >= 0, and 0 for a one-key segment -- the same rule as the greedy fit.

Also: the smallest known case where the greedy fit is not minimal, the fit
never uses more segments than the greedy fit, and the blobs decode.
"""
import numpy as np
import pytest

import oracle
import oracle_pins as P


def test_greedy_is_not_minimal_smallest_case():
    # five keys, eps 3: greedy needs 3 segments, two suffice
    k = np.array([0, 18, 21, 33, 34], np.uint64)
    for F in (0, 4, 20):
        assert len(oracle.fit_block(k, 3, F)[0]) == 3
        st, an, sl = oracle.fit_block(k, 3, F, "min")
        assert len(st) == 2
        if F <= 4:  # the slope brute force grows as 2^F
            best, earliest = P.brute_min_segmentations(k, 3, F)
            assert best == 2 and st.tolist() == earliest[:-1]


def test_min_fit_against_brute_force():
    P.check_min_fit_bruteforce(oracle.default())


def test_min_fit_keys_near_the_cap():
    # anchored slopes stop at D + eps + 1 = 2^(64 - F); both fits obey the cap
    for F in (20, 32):
        top = (1 << 64) - 1
        k = np.array(sorted({0, 5, 1 << 30, (1 << 43) + 7, 1 << 44, top - 3, top}), np.uint64)
        g = oracle.fit_block(k, 3, F)[0]
        m = oracle.fit_block(k, 3, F, "min")[0]
        assert len(m) <= len(g)
        blob = oracle.compress(k, 3, 6, F, fit="min")
        assert np.array_equal(oracle.decode(blob), k)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_min_fit_never_more_segments_and_decodes(seed):
    for keys, eps, log2b in P.random_cases(seed, 10):
        if len(keys) > 20000:
            keys = keys[:20000]
        for F in (0, 20):
            g = oracle.compress(keys, eps, log2b, F)
            m = oracle.compress(keys, eps, log2b, F, fit="min")
            assert oracle.header(m)["nseg_total"] <= oracle.header(g)["nseg_total"]
            assert np.array_equal(oracle.decode(m), keys)
            # every residual of the min fit lies within eps of its prediction
            # (the prediction is reduced modulo 2^(8 key_bytes), as decoding does)
            f = oracle.predict(keys, eps, log2b, F, fit="min")
            mod = 1 << (8 * keys.dtype.itemsize)
            d = [((int(x) - int(y) + mod // 2) % mod) - mod // 2 for x, y in zip(keys, f)]
            assert all(abs(x) <= eps for x in d)


def test_min_fit_equals_greedy_when_greedy_is_one_segment():
    # a block the greedy fit covers with one segment is already minimal
    for g in (0, 1, 3, 1000):
        k = (np.uint64(7) + np.uint64(g) * np.arange(1024, dtype=np.uint64))
        for eps in (0, 7):
            gs = oracle.fit_block(k, eps, 20)
            ms = oracle.fit_block(k, eps, 20, "min")
            assert len(gs[0]) == 1
            assert all(np.array_equal(x, y) for x, y in zip(gs, ms))


def test_min_fit_rejects_unknown_fit():
    with pytest.raises(ValueError):
        oracle.compress(np.arange(10, dtype=np.uint64), 3, fit="optimal")
