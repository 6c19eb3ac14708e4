"""Pins of the oracle's query operators (Sec. III-A list AND / OR, Sec. III-C
quantile and approximate query processing), each against something other
than the function itself:

* predict (the eps-PLA without residuals): the paper's bound |K - f| <= eps;
  exactness on arithmetic progressions; and f + (code - eps) = K with the
  codes read from the oracle's blob by the pins' own bit reader;
* intersect / union: Python set operations on small inputs;
* quantile: numpy's inverted-CDF quantile wherever N*k is not a multiple of
  q (there both are K[floor(N*k/q)]), the edge cases k = 0 and k = q, and
  the median of an odd-length list.
"""
import numpy as np
import pytest

import oracle
import oracle_pins as P


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_predict_error_bound_and_residuals(seed):
    for keys, eps, log2b in P.random_cases(seed, 12):
        if len(keys) > 3000:
            keys = keys[:3000]
        for F in (0, 20, 32):
            f = oracle.predict(keys, eps, log2b, F)
            d = keys.astype(object) - f.astype(object)
            assert max(abs(int(x)) for x in d) <= eps if len(keys) else True
            blob = oracle.compress(keys, eps, log2b, F)
            h = oracle.header(blob)
            B = 1 << log2b
            for b in range(h["nblocks"]):
                nb = min(B, len(keys) - b * B)
                codes = P.read_codes(blob, h, b, nb) if h["width"] else [eps] * nb
                for j in range(nb):
                    i = b * B + j
                    assert int(f[i]) + codes[j] - eps == int(keys[i]), (seed, b, j)


def test_predict_exact_on_arithmetic_progressions():
    for g in (0, 1, 3, 64, 1000, 12345):
        keys = (np.uint64(7) + np.uint64(g) * np.arange(5000, dtype=np.uint64))
        for eps in (0, 7, 255):
            assert np.array_equal(oracle.predict(keys, eps), keys), (g, eps)


def test_set_operations_against_python_sets():
    rng = np.random.default_rng(5)
    for _ in range(200):
        na, nb = int(rng.integers(0, 300)), int(rng.integers(0, 300))
        hi = int(rng.choice([50, 1000, 1 << 40]))
        a = np.sort(rng.integers(0, hi, na).astype(np.uint64))
        b = np.sort(rng.integers(0, hi, nb).astype(np.uint64))
        sa, sb = set(a.tolist()), set(b.tolist())
        assert oracle.intersect(a, b).tolist() == sorted(sa & sb)
        assert oracle.union(a, b).tolist() == sorted(sa | sb)
    u32 = np.array([0, 5, 5, 2 ** 32 - 1], np.uint32)
    assert oracle.intersect(u32, np.array([5, 2 ** 32 - 1], np.uint32)).tolist() == [5, 2 ** 32 - 1]


def test_quantile():
    rng = np.random.default_rng(6)
    for _ in range(100):
        n = int(rng.integers(1, 2000))
        keys = np.sort(rng.integers(0, 1 << 40, n).astype(np.uint64))
        q = int(rng.integers(1, 1000))
        ks = rng.integers(0, q + 1, 20)
        got = oracle.quantile(keys, ks, q)
        for k, v in zip(ks.tolist(), got.tolist()):
            if (n * k) % q and k < q:
                want = np.quantile(keys, k / q, method="inverted_cdf")
                assert v == int(want), (n, k, q)
        assert oracle.quantile(keys, [0], q)[0] == keys[0]
        assert oracle.quantile(keys, [q], q)[0] == keys[-1]
    odd = np.arange(1, 100, 2, dtype=np.uint64)  # 50 keys ... take 49 for an odd length
    odd = odd[:49]
    assert oracle.quantile(odd, [1], 2)[0] == odd[24] == np.median(odd)
