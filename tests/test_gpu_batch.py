"""Batches of lists on the GPU against the CPU oracle, through the C ABI.

A batch gives every list an ordinary blob v1, so the bar is the single-list
one: each list's blob equals the oracle's blob of that list, byte for byte,
and the batch decode returns every list's keys at its offset.  The eps
autotuner must pick, per list, the candidate whose oracle blob is smallest
(ties to the smaller eps), and its size pass must equal the oracle's sizes.
"""
import sys

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
CANDS = (7, 31, 127)


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lc():
    from paper_2412_10770_amd import lc as mod
    return mod


@pytest.fixture(scope="module")
def wl():
    from paper_2412_10770_amd import workloads
    return workloads


def _concat(lists, kb):
    dt = np.uint32 if kb == 4 else np.uint64
    cat = np.concatenate([np.asarray(x, dtype=dt) for x in lists]) if lists else np.zeros(0, dt)
    return torch.from_numpy(cat.view(np.int32 if kb == 4 else np.int64).copy()).to(DEV), cat


def _host(t, kb):
    return t.cpu().numpy().view(np.uint32 if kb == 4 else np.uint64)


def _mixed_lists(rng, kb, count):
    """Lists of every edge length (empty, one key, block +- 1) and gap shape."""
    top = (1 << (8 * kb)) - 1
    lens = [0, 1, 2, 63, 64, 65, 1023, 1024, 1025, 4096, 5000]
    lens += [int(x) for x in rng.integers(1, 6000, count - len(lens))]
    out = []
    for i, n in enumerate(lens):
        kind = i % 5
        if kind == 0:
            gaps = rng.integers(1, 65, n)
        elif kind == 1:
            gaps = rng.geometric(1.0 / float(np.exp(rng.uniform(np.log(2), np.log(2000)))), n)
        elif kind == 2:
            gaps = np.full(n, int(rng.integers(0, 1000)))          # arithmetic progression
        elif kind == 3:
            gaps = rng.integers(0, 3, n)                             # duplicates
        else:
            gaps = rng.integers(0, max(1, top // max(n, 1) // 2), n)  # sparse, wide keys
        start = int(rng.integers(0, 1 << 16))
        keys = start + np.cumsum(gaps.astype(np.uint64), dtype=np.uint64) if n else np.zeros(0, np.uint64)
        keys = np.minimum(keys, np.uint64(top))
        out.append(np.sort(keys).astype(np.uint32 if kb == 4 else np.uint64))
    return out


def _check_batch(lc, batch, lists, eps, log2b, frac_bits, kb, fit="greedy"):
    for l, keys in enumerate(lists):
        want = oracle.compress(keys, int(eps[l]), log2b, frac_bits, fit=fit)
        got = batch.blob(l).data.cpu().numpy()
        assert int(batch.sizes[l]) == len(want), (l, len(keys), int(eps[l]))
        assert np.array_equal(got, want), (l, len(keys), int(eps[l]))
    out = lc.batch_decompress(batch)
    cat = np.concatenate(lists) if lists else np.zeros(0)
    assert np.array_equal(_host(out, kb), cat)


TILINGS = ("rows", "lanes")  # the two wave tilings of the batch fit: identical blobs


@pytest.mark.parametrize("tiling", TILINGS)
@pytest.mark.parametrize("kb,log2b,frac_bits", [(4, 10, 20), (8, 10, 20), (4, 6, 20), (8, 12, 32), (8, 8, 0)])
def test_fixed_eps_per_list(lc, kb, log2b, frac_bits, tiling):
    rng = np.random.default_rng(100 + kb + log2b)
    lists = _mixed_lists(rng, kb, 40)
    eps = rng.choice([0, 1, 7, 31, 63, 127, 1000, 65535], len(lists)).astype(np.uint32)
    _say(f"batch fixed eps kb={kb} log2b={log2b} F={frac_bits} lists={len(lists)} tiling={tiling}")
    keys, _ = _concat(lists, kb)
    batch = lc.batch_compress(keys, [len(x) for x in lists], eps=eps, log2_block=log2b, frac_bits=frac_bits,
                              tiling=tiling)
    assert np.array_equal(batch.eps, eps)
    _check_batch(lc, batch, lists, eps, log2b, frac_bits, kb)
    # a list's blob is an ordinary blob: the single-list queries work on it
    l = max(range(len(lists)), key=lambda i: len(lists[i]))
    b = batch.blob(l)
    idx = torch.from_numpy(rng.integers(0, len(lists[l]), 500).astype(np.int64)).to(DEV)
    assert np.array_equal(_host(lc.access(b, idx), kb), lists[l][idx.cpu().numpy()])


# the better-ratio fits for every list of a batch (Sec. II-A's optimal-L
# goal): per-list blobs equal the oracle's fit of that list
@pytest.mark.parametrize("fit", ["min", "opt"])
@pytest.mark.parametrize("kb,log2b,frac_bits", [(4, 10, 20), (8, 10, 0), (8, 6, 20), (4, 8, 0)])
def test_batch_fits_fixed_eps(lc, fit, kb, log2b, frac_bits):
    rng = np.random.default_rng(300 + kb + log2b + frac_bits)
    lists = _mixed_lists(rng, kb, 24)
    eps = rng.choice([0, 1, 7, 31, 127, 1000], len(lists)).astype(np.uint32)
    _say(f"batch fit={fit} kb={kb} log2b={log2b} F={frac_bits} lists={len(lists)}")
    keys, _ = _concat(lists, kb)
    batch = lc.batch_compress(keys, [len(x) for x in lists], eps=eps, log2_block=log2b, frac_bits=frac_bits, fit=fit)
    assert batch.params.fit == lc.FITS[fit]
    _check_batch(lc, batch, lists, eps, log2b, frac_bits, kb, fit=fit)
    l = max(range(len(lists)), key=lambda i: len(lists[i]))
    b = batch.blob(l)
    assert b.info.flags == (1 if fit == "opt" else 0)
    idx = torch.from_numpy(rng.integers(0, len(lists[l]), 500).astype(np.int64)).to(DEV)
    assert np.array_equal(_host(lc.access(b, idx), kb), lists[l][idx.cpu().numpy()])


@pytest.mark.parametrize("fit", ["min", "opt"])
@pytest.mark.parametrize("frac_bits", [0, 20])
def test_batch_fits_autotune_picks_the_oracle_argmin(lc, fit, frac_bits):
    rng = np.random.default_rng(400 + frac_bits)
    lists = _mixed_lists(rng, 4, 20)
    keys, _ = _concat(lists, 4)
    lengths = [len(x) for x in lists]
    _say(f"batch autotune fit={fit} F={frac_bits} lists={len(lists)}")
    want = np.array([[len(oracle.compress(x, e, 10, frac_bits, fit=fit)) for x in lists] for e in CANDS])
    best = np.array([CANDS[int(np.argmin(want[:, l]))] for l in range(len(lists))], dtype=np.uint32)
    batch = lc.batch_compress(keys, lengths, candidates=CANDS, frac_bits=frac_bits, fit=fit)
    assert np.array_equal(batch.eps, best)
    _check_batch(lc, batch, lists, best, 10, frac_bits, 4, fit=fit)


@pytest.mark.parametrize("tiling", TILINGS)
@pytest.mark.parametrize("kb", [4, 8])
def test_autotune_picks_the_oracle_argmin(lc, kb, tiling):
    rng = np.random.default_rng(200 + kb)
    lists = _mixed_lists(rng, kb, 30)
    _say(f"batch autotune kb={kb} lists={len(lists)} tiling={tiling}")
    keys, _ = _concat(lists, kb)
    lengths = [len(x) for x in lists]
    # the size pass itself
    p, table = lc.batch_plan(lengths, CANDS[0], kb, max(CANDS), frac_bits=20, tiling=tiling)
    d_lists = torch.from_numpy(table.view(np.uint8).copy()).to(DEV)
    ws = torch.empty(p.ws_bytes, dtype=torch.uint8, device=DEV)
    sizes = torch.empty(len(CANDS) * len(lists), dtype=torch.int64, device=DEV)
    stats = torch.zeros(2, dtype=torch.int32, device=DEV)
    lc.batch_sizes_async(keys, d_lists, p, CANDS, ws, sizes, stats)
    got_sizes = sizes.cpu().numpy().reshape(len(CANDS), len(lists))
    assert int(stats[0].item()) == 0
    want_sizes = np.array([[len(oracle.compress(x, e, 10, 20)) for x in lists] for e in CANDS])
    assert np.array_equal(got_sizes, want_sizes)
    best = np.array([CANDS[int(np.argmin(want_sizes[:, l]))] for l in range(len(lists))], dtype=np.uint32)
    batch = lc.batch_compress(keys, lengths, candidates=CANDS, frac_bits=20, tiling=tiling)
    assert np.array_equal(batch.eps, best)
    _check_batch(lc, batch, lists, best, 10, 20, kb)


@pytest.mark.parametrize("tiling", TILINGS)
def test_bad_list_is_flagged_and_skipped(lc, tiling):
    rng = np.random.default_rng(7)
    lists = _mixed_lists(rng, 4, 12)
    keys, _ = _concat(lists, 4)
    lengths = np.array([len(x) for x in lists], dtype=np.uint64)
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.uint64)
    bad = 9
    offs_bad = offs.copy()
    offs_bad[bad] = keys.numel() - lengths[bad] + 1  # one key past the end
    p, table = lc.batch_plan(lengths, 31, 4, frac_bits=20, key_offsets=offs_bad, tiling=tiling)
    d_lists = torch.from_numpy(table.view(np.uint8).copy()).to(DEV)
    ws = torch.empty(p.ws_bytes, dtype=torch.uint8, device=DEV)
    blob = torch.zeros(p.blob_bytes, dtype=torch.uint8, device=DEV)
    sizes = torch.zeros(len(lists), dtype=torch.int64, device=DEV)
    stats = torch.zeros(2, dtype=torch.int32, device=DEV)
    lc.batch_compress_async(keys, d_lists, p, blob, ws, sizes, stats)
    st = stats.cpu().numpy()
    assert st[0] == lc.LC_FLAG_BADLIST
    sz = sizes.cpu().numpy().astype(np.uint64)
    assert sz[bad] == np.uint64(2 ** 64 - 1)
    data = blob.cpu().numpy()
    for l, x in enumerate(lists):
        if l == bad:
            continue
        want = oracle.compress(x, 31, 10, 20)
        o = int(table["blob_off"][l])
        assert np.array_equal(data[o:o + len(want)], want), l
    # decode: the bad list is skipped and flagged, the others land at their offsets
    out = torch.full((keys.numel(),), -1, dtype=torch.int32, device=DEV)
    dstats = torch.zeros(1, dtype=torch.int32, device=DEV)
    lc.batch_decompress_async(blob, d_lists, p, int(st[1]), out, dstats)
    assert int(dstats.item()) == lc.LC_FLAG_BADLIST
    h = _host(out, 4)
    for l, x in enumerate(lists):
        if l != bad:
            assert np.array_equal(h[int(offs[l]):int(offs[l]) + len(x)], x), l


@pytest.mark.parametrize("tiling", TILINGS)
def test_unsorted_list_is_flagged(lc, tiling):
    rng = np.random.default_rng(8)
    lists = _mixed_lists(rng, 8, 12)
    lists[10] = lists[10].copy()  # 5000 keys
    lists[10][100], lists[10][101] = lists[10][101] + 1, lists[10][100]
    keys, _ = _concat(lists, 8)
    with pytest.raises(lc.LcError, match="not sorted"):
        lc.batch_compress(keys, [len(x) for x in lists], eps=15, tiling=tiling)


@pytest.mark.parametrize("tiling", TILINGS)
def test_posting_lists_reduced(lc, wl, tiling):
    """The batch workload's recipe at 256 lists of 100 .. 10^5 keys, autotuned."""
    keys, lengths = wl.posting_lists(256, device=DEV, hi=1e5)
    _say(f"posting lists reduced: {len(lengths)} lists, {keys.numel()} keys, tiling={tiling}")
    batch = lc.batch_compress(keys, lengths, candidates=CANDS, frac_bits=20, tiling=tiling)
    out = lc.batch_decompress(batch)
    assert torch.equal(out, keys)
    host = _host(keys, 4)
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]])
    rng = np.random.default_rng(9)
    for l in sorted(set(rng.choice(len(lengths), 24, replace=False).tolist()) | {int(np.argmax(lengths))}):
        x = host[offs[l]:offs[l] + lengths[l]]
        sizes = [len(oracle.compress(x, e, 10, 20)) for e in CANDS]
        e = CANDS[int(np.argmin(sizes))]
        assert batch.eps[l] == e, l
        assert np.array_equal(batch.blob(l).data.cpu().numpy(), oracle.compress(x, e, 10, 20)), l


@pytest.mark.parametrize("tiling", TILINGS)
def test_tiny_lists_and_degenerate_batches(lc, tiling):
    """20000 lists of 0..3 keys (most work items hold a single block), one
    single-list batch, an all-empty batch, and u64 keys at the top of the
    range: every blob equals the oracle's."""
    rng = np.random.default_rng(31)
    lens = rng.integers(0, 4, 20000)
    top = np.uint64(2 ** 64 - 1)
    lists = []
    for i, m in enumerate(lens):
        base = top - np.uint64(rng.integers(0, 1 << 20)) if i % 7 == 0 else np.uint64(rng.integers(0, 1 << 40))
        x = np.sort(base - rng.integers(0, 1 << 10, m).astype(np.uint64)) if i % 7 == 0 else \
            np.sort(base + rng.integers(0, 1 << 10, m).astype(np.uint64))
        lists.append(x.astype(np.uint64))
    keys, _ = _concat(lists, 8)
    _say("tiny lists: 20000")
    batch = lc.batch_compress(keys, lens, candidates=(0, 5, 1000), tiling=tiling)
    assert torch.equal(lc.batch_decompress(batch), keys)
    for l in rng.choice(len(lists), 300, replace=False):
        sizes = [len(oracle.compress(lists[l], e, 10)) for e in (0, 5, 1000)]
        e = (0, 5, 1000)[int(np.argmin(sizes))]
        assert batch.eps[l] == e
        assert np.array_equal(batch.blob(l).data.cpu().numpy(), oracle.compress(lists[l], e, 10)), l
    # one list
    one = np.cumsum(rng.integers(1, 100, 5000)).astype(np.uint64)
    k1, _ = _concat([one], 8)
    b1 = lc.batch_compress(k1, [len(one)], eps=31, tiling=tiling)
    assert np.array_equal(b1.blob(0).data.cpu().numpy(), oracle.compress(one, 31, 10))
    assert torch.equal(lc.batch_decompress(b1), k1)
    # every list empty: header-only blobs, nothing to decode
    k0 = torch.zeros(0, dtype=torch.int64, device=DEV)
    b0 = lc.batch_compress(k0, [0, 0, 0], eps=7, tiling=tiling)
    for l in range(3):
        assert np.array_equal(b0.blob(l).data.cpu().numpy(), oracle.compress(np.zeros(0, np.uint64), 7, 10))
    assert lc.batch_decompress(b0).numel() == 0


def test_autotune_block_size(lc, wl):
    """The batch autotuner: every block size gives a batch that round-trips
    and whose lists equal the oracle's blobs at that block size; the choice
    is the argmin of the measured objective."""
    keys, lengths = wl.posting_lists(64, device=DEV, hi=2e4)
    _say(f"autotune block size: {keys.numel()} keys")
    best, report = lc.autotune_batch(keys, lengths, block_candidates=(8, 10, 12), objective="size")
    assert sum(r["chosen"] for r in report) == 1
    chosen = next(r for r in report if r["chosen"])
    assert chosen["bytes"] == min(r["bytes"] for r in report)
    assert best.params.log2_block == chosen["log2_block"] and best.nbytes == chosen["bytes"]
    assert torch.equal(lc.batch_decompress(best), keys)
    host = keys.cpu().numpy().view(np.uint32)
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]])
    for l in (0, int(np.argmax(lengths))):
        x = host[offs[l]:offs[l] + lengths[l]]
        want = oracle.compress(x, int(best.eps[l]), chosen["log2_block"])
        assert np.array_equal(best.blob(l).data.cpu().numpy(), want)
    fast, rep2 = lc.autotune_batch(keys, lengths, block_candidates=(8, 12), objective="speed", time_reps=2)
    c2 = next(r for r in rep2 if r["chosen"])
    assert c2["decode_ms"] == min(r["decode_ms"] for r in rep2)


def test_autotune_fit_and_frac_bits(lc, wl):
    """The autotuner's (fit, F) candidates at the chosen block size: the
    choice has the fewest bytes among them, and its lists equal the oracle's
    blobs for that fit and F."""
    keys, lengths = wl.posting_lists(48, device=DEV, hi=2e4)
    _say(f"autotune fit / F: {keys.numel()} keys")
    fits = (("greedy", 0), ("greedy", 20), ("opt", 0), ("opt", 20), ("min", 0))
    best, report = lc.autotune_batch(keys, lengths, block_candidates=(9, 10), objective="size", frac_bits=0,
                                     fit_candidates=fits, tilings=())
    chosen = next(r for r in report if r["chosen"])
    at = [r for r in report if r["log2_block"] == chosen["log2_block"]]
    assert {(r["fit"], r["frac_bits"]) for r in at} == set(fits)
    assert chosen["bytes"] == min(r["bytes"] for r in at)
    assert best.params.fit == lc.FITS[chosen["fit"]] and best.params.frac_bits == chosen["frac_bits"]
    assert torch.equal(lc.batch_decompress(best), keys)
    host = keys.cpu().numpy().view(np.uint32)
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]])
    for l in (0, int(np.argmax(lengths))):
        x = host[offs[l]:offs[l] + lengths[l]]
        want = oracle.compress(x, int(best.eps[l]), chosen["log2_block"], chosen["frac_bits"], fit=chosen["fit"])
        assert np.array_equal(best.blob(l).data.cpu().numpy(), want)


@pytest.mark.parametrize("kb", [4, 8])
def test_batch_and_pairs(lc, kb):
    """AND of many pairs of lists of one batch in one pass: each pair's
    result equals the set intersection of the two lists (either order,
    shared keys, empty lists, a list with itself)."""
    rng = np.random.default_rng(300 + kb)
    dt = np.uint32 if kb == 4 else np.uint64
    base = np.unique(rng.integers(0, 1 << 24, 40000)).astype(dt)
    lists = [np.zeros(0, dt)]
    for i in range(60):
        m = int(rng.integers(1, 6000)) if i % 3 else int(rng.integers(6000, 30000))
        pick = np.sort(rng.choice(base, min(m, len(base)), replace=False)) if i % 4 else \
            np.unique(rng.integers(0, 1 << 24, m)).astype(dt)
        lists.append(pick.astype(dt))
    lists.append(np.sort(rng.integers(0, 300, 4000)).astype(dt))  # duplicates
    keys, _ = _concat(lists, kb)
    batch = lc.batch_compress(keys, [len(x) for x in lists], candidates=CANDS)
    nl = len(lists)
    pairs = [(int(rng.integers(0, nl)), int(rng.integers(0, nl))) for _ in range(500)]
    pairs += [(0, 5), (5, 0), (7, 7), (nl - 1, nl - 1), (nl - 1, 3)]
    _say(f"batch AND kb={kb}: {len(pairs)} pairs of {nl} lists")
    res = lc.batch_intersect(batch, pairs)
    for (a, b), r in zip(pairs, res):
        assert np.array_equal(_host(r, kb), oracle.intersect(lists[a], lists[b])), (a, b)
