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
