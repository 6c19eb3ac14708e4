"""Pins of the oracle's optimal fit (``fit="opt"``: fixed-point lines with a
free intercept, the class of the optimal eps-PLA of Sec. II-A): brute force
over every integer (A, C) on tiny blocks for the boundaries, the minimum
segment count and the stored slope and intercept; closed forms (a line with
a fractional intercept, the cap, intercepts past 2^64); blob decoding and
size.  The checks live in ``oracle_pins`` so the planted-mistake runs use
them too."""
import numpy as np
import pytest

import oracle
import oracle_pins as P


def test_opt_fit_closed_forms():
    P.check_opt_fit_closed_forms(oracle.default())


@pytest.mark.parametrize("seed", [12, 13, 14])
def test_opt_fit_against_brute_force(seed):
    P.check_opt_fit_bruteforce(oracle.default(), trials=600, seed=seed)


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_opt_fit_blobs(seed):
    P.check_opt_fit_blobs(oracle.default(), seed=seed, count=16)


def test_opt_fit_smallest_case():
    # the five-key block where the greedy anchored fit needs three segments
    # and the anchored minimum two: a free intercept does not need fewer here
    k = np.array([0, 18, 21, 33, 34], np.uint64)
    for F in (0, 4, 20):
        st, an, sl, fr = oracle.fit_block(k, 3, F, "opt")
        assert len(st) == 2
        assert len(fr) == 2 and (F > 0 or not fr.any())


def test_opt_fit_never_more_segments_than_anchored_min():
    for keys, eps, log2b in P.random_cases(21, 12):
        keys = keys[:20000]
        for F in (0, 20):
            m = oracle.header(oracle.compress(keys, eps, log2b, F, fit="min"))["nseg_total"]
            o = oracle.header(oracle.compress(keys, eps, log2b, F, fit="opt"))["nseg_total"]
            assert o <= m


def _intercept_window_cases():
    for keys, eps, log2b in P.random_cases(31, 10):
        yield keys, eps, log2b
    rng = np.random.default_rng(31)
    top = np.iinfo(np.uint64).max
    for eps in (0, 3, 255, 1 << 20):
        # ends at 2^64 - 1, alone in the last block (2049 = 8 * 256 + 1):
        # its intercept passes 2^64 for eps >= 2
        gaps = rng.integers(0, 1 << 12, 2049).astype(np.uint64)
        keys = np.uint64(top) - (np.cumsum(gaps[::-1])[::-1] - gaps[-1]).astype(np.uint64)
        yield keys, eps, 8
        yield np.sort(rng.integers(0, 1 << 30, 3000)).astype(np.uint32), eps, 8


@pytest.mark.parametrize("F", [0, 20])
def test_opt_intercepts_within_eps_of_segment_first_keys(F):
    """A free intercept floor(C / 2^F) predicts the segment's first key
    (d = 0), so the eps bound (Def. 2) puts it within eps of that key, and
    C >= first * 2^F puts it at or above the block's first key.  Stored
    modulo 2^64, it wraps only when that key is within eps of 2^64; the
    delta intercept - first is then exact (no wrap) for 4-byte keys and
    whenever first >= eps."""
    M = 1 << 64
    for keys, eps, log2b in _intercept_window_cases():
        B = 1 << log2b
        kb = keys.dtype.itemsize
        for b0 in range(0, len(keys), B):
            blk = keys[b0:b0 + B]
            st, an, _, _ = oracle.fit_block(blk, eps, F, "opt")
            first = int(blk[0])
            for s, a in zip(st.tolist(), an.tolist()):
                ks = int(blk[s])
                cands = [v for v in (int(a), int(a) + M) if abs(v - ks) <= eps]
                assert len(cands) == 1, (b0, s, a, ks, eps)
                icpt = cands[0]
                assert first <= icpt <= ks + eps
                assert icpt < M or ks + eps >= M
                if kb == 4 or first >= eps:
                    delta = (int(a) - first) % M
                    assert delta == icpt - first
                    assert ks - first - eps <= delta <= ks - first + eps
