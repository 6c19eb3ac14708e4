"""Queries on the compressed form against the oracle (Sec. III-A, III-C):
quantiles (exact and from the model alone), the approximate decode (the
eps-PLA without residuals, bit-exact to the oracle's prediction and within
eps of every key), and list AND / OR (the set definitions)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import oracle_pins as P

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lc():
    from paper_2412_10770_amd import lc as mod
    return mod


def _dev(keys):
    return torch.from_numpy(keys.view(np.int32 if keys.dtype.itemsize == 4 else np.int64).copy()).to(DEV)


def _host(t, kb):
    return t.cpu().numpy().view(np.uint32 if kb == 4 else np.uint64)


@pytest.mark.parametrize("seed", [1, 2])
def test_quantile_and_approx_random(lc, seed):
    for keys, eps, log2b in P.random_cases(seed, 14):
        if len(keys) > 3000:
            keys = keys[:3000]
        kb = keys.dtype.itemsize
        n = len(keys)
        for F in (0, 20, 32):
            _say(f"quantile/approx seed={seed} n={n} kb={kb} eps={eps} log2b={log2b} F={F}")
            blob = lc.compress(_dev(keys), eps, log2b, F)
            f = oracle.predict(keys, eps, log2b, F)
            got = _host(lc.decompress_approx(blob), kb)
            assert np.array_equal(got, f)
            d = keys.astype(object) - got.astype(object)
            assert max(abs(int(x)) for x in d) <= eps
            if n > 2:
                a, b = 1, n - 1
                assert np.array_equal(_host(lc.decompress_approx(blob, a, b), kb), f[a:b])
            rng = np.random.default_rng(seed)
            for q in (1, 2, 4, 100, 7919, n):
                ks = np.unique(np.concatenate([[0, q], rng.integers(0, q + 1, 30)])).astype(np.int64)
                kt = torch.from_numpy(ks).to(DEV)
                assert np.array_equal(_host(lc.quantile(blob, kt, q), kb), oracle.quantile(keys, ks, q)), q
                idx = [min((n * int(k)) // q, n - 1) for k in ks]
                assert np.array_equal(_host(lc.quantile(blob, kt, q, approx=True), kb), f[idx]), q


def test_approx_sparse_and_dense_blocks(lc):
    """Blocks whose segment areas are not staged (two-key segments) and
    one-segment blocks; eps 0 gives the keys themselves."""
    rng = np.random.default_rng(9)
    sparse = np.cumsum(rng.integers(1, 1 << 30, 6000)).astype(np.uint64)
    dense = np.cumsum(rng.integers(1, 4, 6000)).astype(np.uint64)
    for keys in (sparse, dense, np.concatenate([dense, dense[-1] + sparse])):
        for eps in (0, 3, 255):
            blob = lc.compress(_dev(keys), eps)
            got = _host(lc.decompress_approx(blob), 8)
            assert np.array_equal(got, oracle.predict(keys, eps))
            if eps == 0:
                assert np.array_equal(got, keys)


def _pair_cases(rng):
    out = []
    for kb in (4, 8):
        dt = np.uint32 if kb == 4 else np.uint64
        top = (1 << (8 * kb)) - 1
        big = np.unique(rng.integers(0, 1 << 22, 200000)).astype(dt)
        small = np.sort(rng.choice(big, 700, replace=False))
        small2 = np.sort(np.concatenate([small[:300], rng.integers(0, 1 << 22, 400).astype(dt)]))
        out.append(("small in big", small2, big))
        out.append(("big vs small", big, small2))
        out.append(("similar", np.unique(rng.integers(0, 1 << 20, 50000)).astype(dt),
                    np.unique(rng.integers(0, 1 << 20, 60000)).astype(dt)))
        out.append(("disjoint", np.arange(0, 5000, dtype=dt), np.arange(100000, 103000, dtype=dt)))
        out.append(("identical", big[:20000], big[:20000].copy()))
        out.append(("one empty", np.zeros(0, dt), big[:3000]))
        out.append(("both empty", np.zeros(0, dt), np.zeros(0, dt)))
        out.append(("duplicates", np.sort(rng.integers(0, 300, 5000)).astype(dt),
                    np.sort(rng.integers(100, 500, 4000)).astype(dt)))
        out.append(("top of range", np.array([0, 5, top - 3, top], dt), np.array([5, top - 1, top], dt)))
        out.append(("tile edges", np.arange(0, 2048, dtype=dt) * 3, np.arange(0, 1025, dtype=dt) * 2))
    return out


def test_intersect_union(lc):
    rng = np.random.default_rng(10)
    for name, a, b in _pair_cases(rng):
        kb = a.dtype.itemsize
        for ea, eb in ((63, 7), (0, 255)):
            _say(f"setop {name} kb={kb} na={len(a)} nb={len(b)} eps={ea}/{eb}")
            A = lc.compress(_dev(a), ea)
            B = lc.compress(_dev(b), eb)
            want_i, want_u = oracle.intersect(a, b), oracle.union(a, b)
            assert np.array_equal(_host(lc.intersect(A, B), kb), want_i), name
            assert np.array_equal(_host(lc.intersect(B, A), kb), want_i), name
            assert np.array_equal(_host(lc.union(A, B), kb), want_u), name
            assert np.array_equal(_host(lc.union(B, A), kb), want_u), name


def test_union_large(lc):
    """OR over several tiles with interleaved and shared keys."""
    rng = np.random.default_rng(11)
    a = np.unique(rng.integers(0, 1 << 40, 300000)).astype(np.uint64)
    b = np.unique(np.concatenate([rng.choice(a, 100000, replace=False),
                                  rng.integers(0, 1 << 40, 200000).astype(np.uint64)]))
    A, B = lc.compress(_dev(a), 63), lc.compress(_dev(b), 255)
    assert np.array_equal(_host(lc.union(A, B), 8), oracle.union(a, b))
    assert np.array_equal(_host(lc.intersect(A, B), 8), oracle.intersect(a, b))


@pytest.mark.parametrize("F", [0, 20])
def test_queries_on_optimal_fit_blobs(lc, F):
    """Quantiles, the model-only decode and list AND / OR on blobs of the
    optimal fit (free intercepts, fraction arrays): the same answers as on
    any blob, and the model-only decode equals the oracle's prediction."""
    rng = np.random.default_rng(30 + F)
    for keys, eps, log2b in P.random_cases(30 + F, 10):
        keys = keys[:4000]
        kb = keys.dtype.itemsize
        n = len(keys)
        _say(f"opt-fit queries n={n} kb={kb} eps={eps} log2b={log2b} F={F}")
        blob = lc.compress(_dev(keys), eps, log2b, F, fit="opt")
        f = oracle.predict(keys, eps, log2b, F, fit="opt")
        assert np.array_equal(_host(lc.decompress_approx(blob), kb), f)
        if n:
            q = 7
            k = torch.arange(q + 1, dtype=torch.int64, device="cuda:0")
            got = _host(lc.quantile(blob, k, q), kb)
            assert np.array_equal(got, oracle.quantile(keys, k.cpu().numpy(), q))
    a = np.unique(rng.integers(0, 1 << 36, 60_000)).astype(np.uint64)
    b = np.unique(np.concatenate([rng.choice(a, 20_000, replace=False),
                                  rng.integers(0, 1 << 36, 40_000).astype(np.uint64)]))
    A = lc.compress(_dev(a), 63, 10, F, fit="opt")
    B = lc.compress(_dev(b), 7, 10, F, fit="opt")
    G = lc.compress(_dev(b), 7)
    assert np.array_equal(_host(lc.intersect(A, B), 8), oracle.intersect(a, b))
    assert np.array_equal(_host(lc.intersect(B, A), 8), oracle.intersect(a, b))
    assert np.array_equal(_host(lc.intersect(A, G), 8), oracle.intersect(a, b))
    assert np.array_equal(_host(lc.union(A, B), 8), oracle.union(a, b))
