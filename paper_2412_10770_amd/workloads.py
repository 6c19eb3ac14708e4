"""Seeded synthetic inputs: sorted integer key lists and query batches.

This module only draws random numbers and sorts them; it holds none of the
compressor's arithmetic, so both the HIP path and the CPU oracle's tests can
use it.  Every generator takes a seed and a torch device; the keys are a
function of (recipe, size, seed, device type) -- the CPU and GPU random
streams differ, so a test always hands the *same* materialised keys to both
sides.

Key lists are returned as 1-D torch tensors holding the unsigned bit
patterns: ``torch.int32`` for 4-byte keys and ``torch.int64`` for 8-byte
keys (``as_numpy`` reinterprets them as uint32/uint64).

Recipes (sizes are parameters; the full sizes are the defaults):

* ``uniform_gaps``: K[0] = 0, gaps i.i.d. uniform integers in [1, 64],
  1,000,000 uint32 keys.
* ``lognormal_distinct``: floor(2^40 * x / M), x ~ lognormal(0, 2), M the
  largest of the first n draws, clipped to 2^40 - 1; sorted and
  de-duplicated, drawing further batches of n/2 until n distinct values
  exist, then exactly n of them picked uniformly (100,000,000 uint64 keys).
* ``heterogeneous_runs``: alternating runs (dense first) whose lengths are
  floor(exp(U[ln lo, ln hi])) with lo, hi = 1e4, 1e6 by default; dense runs
  draw gaps uniform in [1, 4], sparse runs Zipf(1.2) gaps capped at 2^20
  (200,000,000 uint64 keys).
* ``lognormal_gaps``: gaps max(1, ceil(lognormal(3, 1.5))), uint64.
* ``posting_lists``: a batch of uint32 lists shaped like the posting lists
  of an inverted index: 4096 lists whose lengths follow the power law
  P(L) ~ L^-1.1 truncated to [100, 10^6] (inverse CDF, floored; about
  3e8 keys in all), each list starting at 0 with geometric gaps (support
  1, 2, ...) of mean m, m = exp(U[ln 2, ln 2000]) drawn per list.
* ``request_stream``: a serving request stream over a store of n keys:
  Poisson arrivals at a given rate (exponential inter-arrival times; rate
  None = all at time 0), 70% range requests of length
  floor(exp(U[0, ln max_len])) starting uniformly in [0, n - length], 20%
  access(i) with i uniform, 10% lower_bound(q) with q uniform over the key
  range.
* queries: ``uniform_indices`` (i uniform in [0, n)) and ``uniform_keys``
  (q uniform over [lo, hi]).
"""
from __future__ import annotations

import math

import numpy as np
import torch

SEED_BASE = 241210770


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=torch.device(device))
    g.manual_seed(int(seed))
    return g


def as_numpy(keys: torch.Tensor) -> np.ndarray:
    """Host copy of a key tensor as uint32 / uint64."""
    a = keys.detach().cpu().contiguous().numpy()
    return a.view(np.uint32 if a.dtype.itemsize == 4 else np.uint64)


def from_numpy(a: np.ndarray, device="cpu") -> torch.Tensor:
    """Key tensor (int32/int64 bit patterns) from a uint32/uint64 array."""
    a = np.ascontiguousarray(a)
    signed = a.view(np.int32 if a.dtype.itemsize == 4 else np.int64)
    return torch.from_numpy(signed.copy()).to(device)


def uniform_gaps(n: int = 1_000_000, seed: int = SEED_BASE + 1, device="cpu",
                 lo: int = 1, hi: int = 64, key_bytes: int = 4) -> torch.Tensor:
    g = _gen(seed, device)
    if n == 0:
        return torch.zeros(0, dtype=torch.int32 if key_bytes == 4 else torch.int64, device=device)
    gaps = torch.randint(lo, hi + 1, (n,), generator=g, device=device, dtype=torch.int64)
    gaps[0] = 0
    keys = torch.cumsum(gaps, 0)
    return keys.to(torch.int32) if key_bytes == 4 else keys


def lognormal_distinct(n: int = 100_000_000, seed: int = SEED_BASE + 2, device="cpu",
                       sigma: float = 2.0, bits: int = 40) -> torch.Tensor:
    g = _gen(seed, device)
    top = float(2 ** bits)
    first = torch.empty(n, dtype=torch.float64, device=device).log_normal_(0.0, sigma, generator=g)
    M = float(first.max())
    batches = [first]
    while True:
        x = torch.cat(batches)
        v = torch.floor(x * (top / M)).clamp_(max=top - 1).to(torch.int64)
        del x
        u = torch.unique(v, sorted=True)
        del v
        if u.numel() >= n:
            break
        del u
        more = torch.empty(max(n // 2, 1), dtype=torch.float64, device=device)
        more.log_normal_(0.0, sigma, generator=g)
        batches.append(more)
    del batches
    if u.numel() > n:
        pick = torch.randperm(u.numel(), generator=g, device=device)[:n]
        pick, _ = torch.sort(pick)
        u = u[pick]
    return u.contiguous()


def _zipf_gaps(count: int, g: torch.Generator, device, s: float = 1.2,
               cap: int = 1 << 20) -> torch.Tensor:
    """min(Zipf(s), cap) by inverse transform over k = 1 .. cap-1 (the rest -> cap)."""
    from scipy.special import zeta
    k = torch.arange(1, cap, dtype=torch.float64, device=device)
    pmf = k.pow(-s) / float(zeta(s, 1))
    cdf = torch.cumsum(pmf, 0)
    u = torch.rand(count, dtype=torch.float64, device=device, generator=g)
    idx = torch.searchsorted(cdf, u, right=True)  # number of k with cdf <= u
    return (idx + 1).clamp_(max=cap).to(torch.int64)


def heterogeneous_runs(n: int = 200_000_000, seed: int = SEED_BASE + 3, device="cpu",
                       run_lo: float = 1e4, run_hi: float = 1e6) -> torch.Tensor:
    g = _gen(seed, device)
    gaps = torch.empty(n, dtype=torch.int64, device=device)
    pos, dense = 0, True
    while pos < n:
        u = float(torch.rand(1, generator=g, dtype=torch.float64, device=device))
        length = int(math.floor(math.exp(math.log(run_lo) + u * (math.log(run_hi) - math.log(run_lo)))))
        length = max(1, min(length, n - pos))
        if dense:
            gaps[pos:pos + length] = torch.randint(1, 5, (length,), generator=g, device=device)
        else:
            gaps[pos:pos + length] = _zipf_gaps(length, g, device)
        pos += length
        dense = not dense
    gaps[0] = 0
    return torch.cumsum(gaps, 0)


def lognormal_gaps(n: int, seed: int = SEED_BASE + 5, device="cpu", mu: float = 3.0,
                   sigma: float = 1.5) -> torch.Tensor:
    g = _gen(seed, device)
    x = torch.empty(n, dtype=torch.float64, device=device).log_normal_(mu, sigma, generator=g)
    gaps = torch.ceil(x).clamp_(min=1).to(torch.int64)
    if n:
        gaps[0] = 0
    return torch.cumsum(gaps, 0)


def posting_lengths(nlists: int = 4096, seed: int = SEED_BASE + 6, lo: float = 100, hi: float = 1e6,
                    s: float = 1.1) -> np.ndarray:
    """List lengths from the power law L^-s truncated to [lo, hi] (inverse CDF, floored)."""
    rng = np.random.default_rng(seed)
    u = rng.random(nlists)
    a = 1.0 - s
    x = (lo ** a + u * (hi ** a - lo ** a)) ** (1.0 / a)
    return np.clip(np.floor(x), lo, hi).astype(np.int64)


def posting_lists(nlists: int = 4096, seed: int = SEED_BASE + 6, device="cpu", lo: float = 100,
                  hi: float = 1e6, s: float = 1.1, mean_lo: float = 2.0, mean_hi: float = 2000.0):
    """(keys, lengths): the lists stored one after another as one uint32 key
    tensor (int32 bit patterns), and the host array of their lengths."""
    lengths = posting_lengths(nlists, seed, lo, hi, s)
    rng = np.random.default_rng(seed + 1)
    means = np.exp(rng.uniform(math.log(mean_lo), math.log(mean_hi), nlists))
    n = int(lengths.sum())
    g = _gen(seed + 2, device)
    lens_t = torch.from_numpy(lengths).to(device)
    # per-key log(1 - p), p = 1 / m, for inverse-CDF geometric draws
    lq = torch.from_numpy(np.log1p(-1.0 / means)).to(device).repeat_interleave(lens_t)
    u = torch.rand(n, dtype=torch.float64, device=device, generator=g)
    gaps = torch.floor(torch.log1p(-u) / lq).to(torch.int64) + 1
    del u, lq
    starts = torch.cumsum(lens_t, 0) - lens_t
    gaps[starts[lengths > 0]] = 0  # every list starts at 0
    keys = torch.cumsum(gaps, 0)
    del gaps
    # restart the running sum at each list
    base = keys[starts[lengths > 0]]
    keys -= base.repeat_interleave(lens_t[lengths > 0])
    if n and int(keys.max()) >= 1 << 32:
        raise ValueError("a list exceeds the uint32 key range")
    return keys.to(torch.int32), lengths


def request_stream(count: int, n: int, key_lo: int, key_hi: int, qps: float | None, seed: int,
                   max_len: int = 1_000_000, mix=(0.7, 0.2, 0.1)):
    """(op, a, b, arrival_ns) numpy arrays; op 1 = range [a, b), 2 = access(a),
    3 = lower_bound(a)."""
    rng = np.random.default_rng(seed)
    u = rng.random(count)
    op = np.where(u < mix[0], 1, np.where(u < mix[0] + mix[1], 2, 3)).astype(np.uint32)
    a = np.zeros(count, dtype=np.uint64)
    b = np.zeros(count, dtype=np.uint64)
    rl = np.floor(np.exp(rng.uniform(0.0, math.log(max_len), count))).astype(np.int64)
    rl = np.minimum(np.maximum(rl, 1), n)
    start = (rng.random(count) * (n - rl + 1)).astype(np.int64)
    rng_ = op == 1
    a[rng_] = start[rng_]
    b[rng_] = (start + rl)[rng_]
    acc = op == 2
    a[acc] = rng.integers(0, n, int(acc.sum()))
    lb = op == 3
    a[lb] = rng.integers(key_lo, key_hi + 1, int(lb.sum()), dtype=np.uint64)
    if qps is None:
        arrival = np.zeros(count, dtype=np.uint64)
    else:
        arrival = np.cumsum(rng.exponential(1e9 / qps, count)).astype(np.uint64)
    return op, a, b, arrival


def uniform_indices(m: int, n: int, seed: int, device="cpu") -> torch.Tensor:
    g = _gen(seed, device)
    if n == 0:
        return torch.zeros(m, dtype=torch.int64, device=device)
    return torch.randint(0, n, (m,), generator=g, device=device, dtype=torch.int64)


def uniform_keys(m: int, lo: int, hi: int, seed: int, device="cpu", key_bytes: int = 8) -> torch.Tensor:
    """q uniform over the integers [lo, hi] (hi - lo < 2^63)."""
    g = _gen(seed, device)
    span = hi - lo + 1
    if span <= 2 ** 62:
        q = torch.randint(0, span, (m,), generator=g, device=device, dtype=torch.int64) + lo
    else:
        r = torch.rand(m, dtype=torch.float64, generator=g, device=device)
        q = (r * float(span)).to(torch.int64) + lo
    return q.to(torch.int32) if key_bytes == 4 else q


def edge_lists():
    """Small hand-made key lists for edge cases: (name, uint array)."""
    out = []
    out.append(("empty_u32", np.zeros(0, np.uint32)))
    out.append(("single_u64", np.array([12345678901234], np.uint64)))
    out.append(("all_equal", np.full(3000, 7, np.uint32)))
    out.append(("max_u32", (np.uint64(2**32 - 1) - np.arange(2500, dtype=np.uint64)[::-1] * 3)
                .astype(np.uint32)))
    out.append(("max_u64", np.uint64(2**64 - 1) - np.arange(2500, dtype=np.uint64)[::-1] * np.uint64(5)))
    huge = np.cumsum(np.full(2100, 1 << 45, dtype=np.uint64))  # gaps beyond the cap at F = 20
    out.append(("cap_gaps", huge))
    return out
