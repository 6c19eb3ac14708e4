"""HIP path against the CPU oracle, through the C ABI.

Integer work, so the bar is bit-exact everywhere: the GPU blob equals the
oracle's blob byte for byte, each side decodes the other's blob to K, and
decompress_range / access / lower_bound equal the plain definitions
(K[b:e], K[i], numpy.searchsorted(..., 'left')).
"""
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


@pytest.fixture(scope="module")
def wl():
    from paper_2412_10770_amd import workloads
    return workloads


def _to_dev(keys: np.ndarray) -> torch.Tensor:
    signed = keys.view(np.int32 if keys.dtype.itemsize == 4 else np.int64)
    return torch.from_numpy(signed.copy()).to(DEV)


def _host(t: torch.Tensor, kb: int) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32 if kb == 4 else np.uint64)


def check_all(lc, keys: np.ndarray, eps: int, log2b: int, rng, nq: int = 2000, frac_bits: int = 20,
              fit: str = "greedy"):
    kb = keys.dtype.itemsize
    n = len(keys)
    _say(f"case n={n} kb={kb} eps={eps} log2b={log2b} F={frac_bits} fit={fit}")
    want = oracle.compress(keys, eps, log2b, frac_bits, fit=fit)
    d = _to_dev(keys)
    blob = lc.compress(d, eps, log2b, frac_bits, fit=fit)
    got = blob.data.cpu().numpy()
    if not np.array_equal(got, want):
        h = oracle.header(want)
        first = int(np.flatnonzero(got[:len(want)] != want[:len(got)])[0]) if min(len(got), len(want)) else -1
        raise AssertionError(f"blob mismatch: sizes {len(got)} vs {len(want)}, first byte {first}, header {h}")
    # both decoders on both blobs
    assert np.array_equal(_host(lc.decompress(blob), kb), keys)
    assert np.array_equal(oracle.decode(got), keys)
    ob = lc.Blob.from_device(torch.from_numpy(want).to(DEV))
    assert np.array_equal(_host(lc.decompress(ob), kb), keys)
    if n == 0:
        return blob
    # ranges: aligned, unaligned, single key, whole list
    ranges = [(0, n), (0, 1), (n - 1, n)]
    for _ in range(6):
        a = int(rng.integers(0, n))
        b = int(rng.integers(a, n + 1))
        ranges.append((a, b))
    for a, b in ranges:
        assert np.array_equal(_host(lc.decompress_range(blob, a, b), kb), keys[a:b]), (a, b)
    # access
    idx = rng.integers(0, n, nq).astype(np.int64)
    idx[:3] = [0, n - 1, n // 2]
    acc = lc.access(blob, torch.from_numpy(idx).to(DEV))
    assert np.array_equal(_host(acc, kb), oracle.access(keys, idx))
    # lower_bound: keys, neighbours, extremes, random
    top = (1 << (8 * kb)) - 1
    cand = [0, top, int(keys[0]), int(keys[-1])]
    cand += [int(x) for x in keys[rng.integers(0, n, nq // 4)]]
    cand += [min(top, int(x) + 1) for x in keys[rng.integers(0, n, nq // 4)]]
    cand += [max(0, int(x) - 1) for x in keys[rng.integers(0, n, nq // 4)]]
    # eps and 2 eps away: the edges of the window in which a free intercept
    # leaves the segment search undecided
    for off in (eps, eps + 1, 2 * eps, 2 * eps + 1):
        cand += [min(top, int(x) + off) for x in keys[rng.integers(0, n, nq // 8)]]
        cand += [max(0, int(x) - off) for x in keys[rng.integers(0, n, nq // 8)]]
    lo, hi = int(keys[0]), int(keys[-1])
    cand += [lo + int(v) for v in rng.integers(0, max(1, min(hi - lo + 1, 2 ** 62)), nq // 4)]
    q = np.array(cand, dtype=keys.dtype)
    pos = lc.lower_bound(blob, _to_dev(q)).cpu().numpy().astype(np.uint64)
    assert np.array_equal(pos, oracle.lower_bound(keys, q))
    return blob


def test_random_small_cases(lc):
    rng = np.random.default_rng(11)
    for keys, eps, log2b in P.random_cases(seed=21, count=50):
        check_all(lc, keys, eps, log2b, rng)


@pytest.mark.parametrize("frac_bits", [0, 8, 32])
def test_other_frac_bits(lc, frac_bits):
    rng = np.random.default_rng(frac_bits)
    for keys, eps, log2b in P.random_cases(seed=30 + frac_bits, count=8):
        check_all(lc, keys, eps, log2b, rng, frac_bits=frac_bits)


def test_edge_lists(lc, wl):
    rng = np.random.default_rng(12)
    for name, keys in wl.edge_lists():
        for eps in (0, 1, 63, 2 ** 31 - 1):
            for log2b in (6, 10, 12):
                check_all(lc, keys, eps, log2b, rng, nq=200)


def test_golden_blobs_on_gpu(lc):
    for name in ("ap4_eps1.txt", "break4_eps1.txt", "opt4_frac_eps0.txt"):
        g = P.load_golden(name)
        keys = np.array(g["keys"], np.uint32 if g["key_bytes"] == 4 else np.uint64)
        blob = lc.compress(_to_dev(keys), g["eps"], g["log2_block"], g["frac_bits"], fit=g.get("fit", "greedy"))
        assert np.array_equal(blob.data.cpu().numpy(), g["blob"]), name
        assert np.array_equal(_host(lc.decompress(blob), g["key_bytes"]), keys), name


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1023, 1024, 1025, 4096 * 3 + 5])
def test_block_edges(lc, n):
    rng = np.random.default_rng(n)
    keys = np.cumsum(rng.integers(1, 65, n)).astype(np.uint64)
    for log2b in (6, 10, 12):
        check_all(lc, keys, 63, log2b, rng, nq=300)


def test_long_segments_and_singletons(lc):
    rng = np.random.default_rng(5)
    ap = (np.uint64(3) + np.uint64(17) * np.arange(50_000, dtype=np.uint64))
    check_all(lc, ap, 0, 12, rng)           # one segment per 4096-key block
    cap = np.cumsum(np.full(9000, 1 << 45, dtype=np.uint64))
    check_all(lc, cap, 3, 12, rng)          # every key its own segment
    check_all(lc, np.full(10_000, 123, np.uint32), 5, 10, rng)


def test_determinism(lc):
    rng = np.random.default_rng(1)
    keys = np.cumsum(rng.integers(0, 1000, 300_000)).astype(np.uint64)
    d = _to_dev(keys)
    a = lc.compress(d, 63).data
    b = lc.compress(d, 63).data
    assert torch.equal(a, b)


def test_unsorted_flag(lc):
    keys = np.arange(5000, dtype=np.uint64) * np.uint64(7) + np.uint64(10)
    for pos in (0, 1, 1023, 1024, 2500, 4999):
        bad = keys.copy()
        if pos == 0:
            bad[0] = bad[1] + np.uint64(1)
        else:
            bad[pos] = bad[pos - 1] - np.uint64(1)  # one key below its predecessor (keys start at 10: no wrap)
        assert bad[pos] != keys[pos] and not np.all(np.diff(bad.astype(np.int64)) >= 0)
        assert np.flatnonzero(np.diff(bad.astype(np.int64)) < 0)[0] in (pos - 1, pos)
        with pytest.raises(lc.LcError):
            lc.compress(_to_dev(bad), 15)


def test_access_out_of_range_flag(lc):
    keys = np.arange(3000, dtype=np.uint32) * np.uint32(5)
    blob = lc.compress(_to_dev(keys), 7)
    idx = torch.tensor([0, 2999, 3000, 2 ** 40], dtype=torch.int64, device=DEV)
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    out = lc.access(blob, idx, flags=flags)
    assert int(flags.item()) == lc.LC_FLAG_RANGE
    assert out.cpu().tolist() == [0, 2999 * 5, 0, 0]
    with pytest.raises(lc.LcError):
        lc.access(blob, idx)


def test_point_queries_beyond_one_per_thread(lc, wl):
    """More queries than threads in one launch (2^24 + 4099): threads past
    the first pass loop to a second query.  access (with one index out of
    range, last), lower_bound and quantiles against the plain definitions;
    quantiles on the threads' second queries plus a random sample."""
    rng = np.random.default_rng(7)
    keys = wl.as_numpy(wl.lognormal_distinct(1_000_000, device="cpu"))
    n = len(keys)
    m = (1 << 24) + 4099
    _say(f"point queries m={m} n={n}")
    blob = lc.compress(_to_dev(keys), 63, 10, 0)
    idx = rng.integers(0, n, m).astype(np.int64)
    idx[-1] = n  # out of range: flagged, answered 0
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    acc = _host(lc.access(blob, torch.from_numpy(idx).to(DEV), flags=flags, check=False), 8)
    assert int(flags.item()) == lc.LC_FLAG_RANGE
    assert acc[-1] == 0 and np.array_equal(acc[:-1], oracle.access(keys, idx[:-1]))
    lo, hi = int(keys[0]), int(keys[-1])
    q = (lo + rng.integers(0, hi - lo + 2, m)).astype(np.uint64)
    pos = lc.lower_bound(blob, _to_dev(q)).cpu().numpy().astype(np.uint64)
    assert np.array_equal(pos, oracle.lower_bound(keys, q))
    qq = 1_000_003
    ks = rng.integers(0, qq + 1, m).astype(np.int64)
    got = _host(lc.quantile(blob, torch.from_numpy(ks).to(DEV), qq), 8)
    sel = np.concatenate([np.arange((1 << 24) - 64, m), rng.integers(0, m, 20_000)])
    assert np.array_equal(got[sel], oracle.quantile(keys, ks[sel], qq))


def test_configs_reduced(lc, wl):
    """The benchmark recipes at sizes the oracle finishes in seconds."""
    rng = np.random.default_rng(2)
    keys = wl.as_numpy(wl.uniform_gaps(1_000_000, device="cpu"))
    check_all(lc, keys, 63, 10, rng, nq=100_000)  # the 1M uint32 workload, at full size
    keys = wl.as_numpy(wl.lognormal_distinct(2_000_000, device="cpu"))
    for eps in (15, 63, 255):
        check_all(lc, keys, eps, 10, rng, nq=20_000)
    keys = wl.as_numpy(wl.heterogeneous_runs(2_000_000, device="cpu", run_lo=1e3, run_hi=1e5))
    check_all(lc, keys, 63, 10, rng, nq=20_000)
    keys = wl.as_numpy(wl.lognormal_gaps(2_000_000, device="cpu"))
    for eps in (255, 1023):
        check_all(lc, keys, eps, 10, rng, nq=20_000)


def _width_combo_lists():
    """Lists whose 64-key blocks cover all 16 (anchor bytes, slope bytes) pairs."""
    rng = np.random.default_rng(0)
    out = []
    for _ in range(400):
        F = int(rng.choice([0, 4, 12, 20]))
        eps = int(rng.choice([0, 1, 7, 255]))
        scale = int(rng.choice([0, 1, 3, 8, 16, 24, 33, 40]))
        gaps = rng.integers(0, 2 ** scale + 1, 512).astype(np.uint64)
        if rng.random() < 0.3:
            gaps[rng.random(512) < 0.05] = np.uint64(2 ** int(rng.integers(20, 46)))
        out.append((np.cumsum(gaps).astype(np.uint64), eps, F))
    out.append((np.arange(0, 64 * 5000, 5000, dtype=np.uint64), 0, 20))
    out.append((np.concatenate([np.arange(0, 3 * 4100, 4100),
                                30000 + np.arange(0, 61 * 4100, 4100)]).astype(np.uint64), 0, 20))
    return out


def test_width_combinations(lc):
    """Decode has a specialised loop per (anchor, slope) byte width; cover all 16."""
    rng = np.random.default_rng(9)
    seen = set()
    for keys, eps, F in _width_combo_lists():
        blob = oracle.compress(keys, eps, 6, F)
        h = oracle.header(blob)
        d = blob[h["off_dir"]:h["off_dir"] + 16 * h["nblocks"]].reshape(-1, 16)
        seen |= set(zip(d[:, 14].tolist(), d[:, 15].tolist()))
        check_all(lc, keys, eps, 6, rng, nq=64, frac_bits=F)
    assert seen == {(a, s) for a in (1, 2, 4, 8) for s in (1, 2, 4, 8)}, sorted(seen)


@pytest.mark.parametrize("kb", [4, 8])
def test_outputs_at_any_key_offset(lc, kb):
    """Decoded keys go to outputs aligned only to the key width: every group
    of keys is stored where its output address is 16-byte aligned, the rest
    key by key."""
    rng = np.random.default_rng(40 + kb)
    keys = np.cumsum(rng.integers(1, 300, 20_000)).astype(np.uint32 if kb == 4 else np.uint64)
    d = _to_dev(keys)
    blob = lc.compress(d, 31)
    n = len(keys)
    dt = torch.int32 if kb == 4 else torch.int64
    for shift in range(16 // kb):
        _say(f"output shift {shift} kb={kb}")
        buf = torch.full((n + 8,), -1, dtype=dt, device=DEV)
        out = buf[shift:shift + n]
        lc.decompress(blob, out=out)
        h = _host(buf, kb)
        assert np.array_equal(h[shift:shift + n], keys)
        assert np.all(h[:shift] == h.dtype.type(-1 & ((1 << (8 * kb)) - 1)))
        assert np.all(h[shift + n:] == h.dtype.type(-1 & ((1 << (8 * kb)) - 1)))
        for a, b in ((1, 1030), (3, n), (1024, 2049), (5, 6), (n - 7, n)):
            buf.fill_(-1)
            lc.decompress_range(blob, a, b, out=buf[shift:shift + b - a])
            h = _host(buf, kb)
            assert np.array_equal(h[shift:shift + b - a], keys[a:b]), (shift, a, b)
            assert np.all(h[shift + b - a:] == h.dtype.type(-1 & ((1 << (8 * kb)) - 1))), (shift, a, b)


@pytest.mark.parametrize("kb", [4, 8])
def test_sparse_blocks_read_from_global(lc, kb):
    """Blocks whose segment area exceeds the 4 KB staged in LDS (about two
    keys per segment) are decoded with the model arrays read from the blob:
    full decode, ranges at every output phase, and a batch of such lists at
    odd key offsets, all against the oracle's blob and the keys."""
    rng = np.random.default_rng(60 + kb)
    top = (1 << (8 * kb)) - 1
    n = 9000
    gaps = rng.integers(1, top // (2 * n), n).astype(np.uint64)
    gaps[rng.random(n) < 0.3] = 1  # mixed with dense stretches
    keys = np.cumsum(gaps, dtype=np.uint64).astype(np.uint32 if kb == 4 else np.uint64)
    _say(f"sparse blocks kb={kb}")
    blob = check_all(lc, keys, 3, 10, rng, nq=500)
    h = blob.info
    data = blob.data.cpu().numpy()
    dirs = data[h.off_dir:h.off_dir + 16 * h.nblocks].reshape(-1, 16)
    ns = dirs[:, 8:12].copy().view(np.uint32).ravel().astype(np.int64)
    area = (2 * ns + 15) // 16 * 16 + (dirs[:, 14] * ns + 15) // 16 * 16 + (dirs[:, 15] * ns + 15) // 16 * 16
    assert (area > 4096).sum() >= 2, "the case must contain blocks that are not staged"
    dt = torch.int32 if kb == 4 else torch.int64
    for shift in range(16 // kb):
        buf = torch.full((n + 8,), -1, dtype=dt, device=DEV)
        for a, b in ((1, n), (1023, 3077), (2 + shift, n - 1)):
            lc.decompress_range(blob, a, b, out=buf[shift:shift + b - a])
            assert np.array_equal(_host(buf, kb)[shift:shift + b - a], keys[a:b]), (shift, a, b)
    # batch: three copies at odd offsets (lists after a 1-key and a 3-key list)
    lists = [keys[:1], keys, keys[:3], keys, keys[5:]]
    cat = np.concatenate(lists)
    d = _to_dev(cat)
    batch = lc.batch_compress(d, [len(x) for x in lists], eps=3)
    assert np.array_equal(_host(lc.batch_decompress(batch), kb), cat)
    assert np.array_equal(batch.blob(1).data.cpu().numpy(), oracle.compress(keys, 3, 10))


@pytest.mark.parametrize("frac_bits", [0, 20, 32])
def test_short_and_long_segments_alternate(lc, frac_bits):
    """Stretches of two- and three-key segments (the fit's short-segment
    step) alternating with long arithmetic runs (its ordinary step), with
    gaps that trigger the overflow cap inside the sparse stretches."""
    rng = np.random.default_rng(70 + frac_bits)
    parts, pos = [], np.uint64(5)
    cap_gap = np.uint64(1) << np.uint64(64 - frac_bits) if frac_bits else np.uint64(0)  # D + eps + 1 >= 2^(64-F)
    for k in range(60):
        if k % 2 == 0:  # long arithmetic run
            m, g = int(rng.integers(5, 400)), int(rng.integers(0, 50))
            run = pos + np.uint64(g) * np.arange(m, dtype=np.uint64)
        else:  # sparse: random wide gaps, sometimes past the cap
            m = int(rng.integers(3, 300))
            gaps = rng.integers(1, 1 << 30, m).astype(np.uint64)
            if frac_bits and k % 6 == 1:
                gaps[rng.integers(0, m)] = cap_gap
            run = pos + np.cumsum(gaps, dtype=np.uint64)
        parts.append(run)
        pos = run[-1] + np.uint64(1)
        if pos > np.uint64(1) << np.uint64(62):
            break
    keys = np.concatenate(parts)
    assert np.all(np.diff(keys.astype(object)) >= 0)
    for eps in (0, 3, 100):
        for log2b in (6, 10):
            check_all(lc, keys, eps, log2b, rng, nq=300, frac_bits=frac_bits)


# --- fewest-segment fit (fit="min"): same blob format, other boundaries --------

def test_min_fit_random_small_cases(lc):
    rng = np.random.default_rng(41)
    for keys, eps, log2b in P.random_cases(seed=41, count=40):
        check_all(lc, keys, eps, log2b, rng, nq=300, fit="min")


@pytest.mark.parametrize("frac_bits", [0, 8, 32])
def test_min_fit_other_frac_bits(lc, frac_bits):
    rng = np.random.default_rng(50 + frac_bits)
    for keys, eps, log2b in P.random_cases(seed=50 + frac_bits, count=8):
        check_all(lc, keys, eps, log2b, rng, nq=200, frac_bits=frac_bits, fit="min")


def test_min_fit_edge_lists(lc, wl):
    rng = np.random.default_rng(13)
    for name, keys in wl.edge_lists():
        for eps in (0, 63, 2 ** 31 - 1):
            for log2b in (6, 12):
                check_all(lc, keys, eps, log2b, rng, nq=100, fit="min")


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 1025, 4096 * 3 + 5])
def test_min_fit_block_edges(lc, n):
    rng = np.random.default_rng(100 + n)
    keys = np.cumsum(rng.integers(1, 65, n)).astype(np.uint64)
    for log2b in (6, 10, 12):
        check_all(lc, keys, 31, log2b, rng, nq=200, fit="min")


def test_min_fit_long_segments_and_singletons(lc):
    """One segment per block (an anchor reaching the block's end early, so
    later anchors are skipped), every key its own segment, equal keys."""
    rng = np.random.default_rng(6)
    ap = (np.uint64(3) + np.uint64(17) * np.arange(50_000, dtype=np.uint64))
    check_all(lc, ap, 0, 12, rng, nq=200, fit="min")
    cap = np.cumsum(np.full(9000, 1 << 45, dtype=np.uint64))
    check_all(lc, cap, 3, 12, rng, nq=200, fit="min")
    check_all(lc, np.full(10_000, 123, np.uint32), 5, 10, rng, nq=200, fit="min")
    # dense block: every anchor's cone stays open for hundreds of keys
    dense = np.cumsum(rng.integers(0, 3, 3 * 4096 + 17)).astype(np.uint32)
    check_all(lc, dense, 255, 12, rng, nq=200, fit="min")


@pytest.mark.parametrize("frac_bits", [0, 20, 32])
def test_min_fit_short_and_long_segments_alternate(lc, frac_bits):
    rng = np.random.default_rng(90 + frac_bits)
    parts, pos = [], np.uint64(5)
    cap_gap = np.uint64(1) << np.uint64(64 - frac_bits) if frac_bits else np.uint64(0)
    for k in range(40):
        if k % 2 == 0:
            m, g = int(rng.integers(5, 400)), int(rng.integers(0, 50))
            run = pos + np.uint64(g) * np.arange(m, dtype=np.uint64)
        else:
            m = int(rng.integers(3, 300))
            gaps = rng.integers(1, 1 << 30, m).astype(np.uint64)
            if frac_bits and k % 6 == 1:
                gaps[rng.integers(0, m)] = cap_gap
            run = pos + np.cumsum(gaps, dtype=np.uint64)
        parts.append(run)
        pos = run[-1] + np.uint64(1)
        if pos > np.uint64(1) << np.uint64(62):
            break
    keys = np.concatenate(parts)
    for eps in (0, 3, 100):
        for log2b in (6, 10):
            check_all(lc, keys, eps, log2b, rng, nq=200, frac_bits=frac_bits, fit="min")


def test_min_fit_width_combinations(lc):
    rng = np.random.default_rng(19)
    for keys, eps, F in _width_combo_lists()[::4]:
        check_all(lc, keys, eps, 6, rng, nq=32, frac_bits=F, fit="min")


def test_min_fit_configs_reduced(lc, wl):
    """The benchmark recipes at sizes the oracle's fewest-segment fit
    finishes in seconds."""
    rng = np.random.default_rng(3)
    keys = wl.as_numpy(wl.uniform_gaps(1_000_000, device="cpu"))
    check_all(lc, keys, 31, 10, rng, nq=20_000, fit="min")
    keys = wl.as_numpy(wl.lognormal_distinct(1_000_000, device="cpu"))
    for eps in (15, 255):
        check_all(lc, keys, eps, 10, rng, nq=20_000, fit="min")
    keys = wl.as_numpy(wl.heterogeneous_runs(300_000, device="cpu", run_lo=1e3, run_hi=1e5))
    check_all(lc, keys, 63, 10, rng, nq=20_000, fit="min")
    keys = wl.as_numpy(wl.lognormal_gaps(1_000_000, device="cpu"))
    check_all(lc, keys, 255, 10, rng, nq=20_000, fit="min")


def test_min_fit_determinism_and_unsorted(lc):
    rng = np.random.default_rng(2)
    keys = np.cumsum(rng.integers(0, 1000, 300_000)).astype(np.uint64)
    d = _to_dev(keys)
    assert torch.equal(lc.compress(d, 63, fit="min").data, lc.compress(d, 63, fit="min").data)
    g, m = lc.compress(d, 63), lc.compress(d, 63, fit="min")
    assert m.info.nseg_total <= g.info.nseg_total
    bad = keys[:5000].copy()
    bad[2500] = bad[2499] - np.uint64(1)
    with pytest.raises(lc.LcError):
        lc.compress(_to_dev(bad), 15, fit="min")


# --- optimal fit (fit="opt"): free fixed-point intercept, fraction array ------

def test_opt_fit_random_small_cases(lc):
    rng = np.random.default_rng(61)
    for keys, eps, log2b in P.random_cases(seed=61, count=40):
        check_all(lc, keys, eps, log2b, rng, nq=300, fit="opt")


@pytest.mark.parametrize("frac_bits", [0, 5, 12, 32])
def test_opt_fit_other_frac_bits(lc, frac_bits):
    """F = 0 (no fraction array), 1-, 2- and 4-byte fractions."""
    rng = np.random.default_rng(70 + frac_bits)
    for keys, eps, log2b in P.random_cases(seed=70 + frac_bits, count=10):
        check_all(lc, keys, eps, log2b, rng, nq=200, frac_bits=frac_bits, fit="opt")


def test_opt_fit_edge_lists(lc, wl):
    rng = np.random.default_rng(14)
    for name, keys in wl.edge_lists():
        for eps in (0, 63, 2 ** 31 - 1):
            for log2b in (6, 12):
                check_all(lc, keys, eps, log2b, rng, nq=100, fit="opt")


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 1025, 4096 * 3 + 5])
def test_opt_fit_block_edges(lc, n):
    rng = np.random.default_rng(200 + n)
    keys = np.cumsum(rng.integers(1, 65, n)).astype(np.uint64)
    for log2b in (6, 10, 12):
        check_all(lc, keys, 31, log2b, rng, nq=200, fit="opt")


def test_opt_fit_lines_caps_and_top_of_range(lc):
    """A fixed-point line with a fractional intercept (one segment per block
    at eps 0), one long segment per block with large hulls, two-key segments
    at the cap, equal keys, and keys at the top of the 64-bit range, where
    intercepts pass 2^64 and are stored modulo 2^64."""
    rng = np.random.default_rng(7)
    line = np.array([(1000 * 256 + 77 + 700 * i) >> 8 for i in range(40_000)], np.uint64)
    blob = check_all(lc, line, 0, 10, rng, nq=200, frac_bits=8, fit="opt")
    assert blob.info.nseg_total == -(-len(line) // 1024)
    dense = np.cumsum(rng.integers(0, 3, 3 * 4096 + 17)).astype(np.uint32)
    check_all(lc, dense, 255, 12, rng, nq=200, fit="opt")
    cap = np.cumsum(np.full(9000, 1 << 45, dtype=np.uint64))
    check_all(lc, cap, 3, 12, rng, nq=200, fit="opt")
    check_all(lc, np.full(10_000, 123, np.uint32), 5, 10, rng, nq=200, fit="opt")
    top = np.uint64((1 << 64) - 1)
    high = top - np.cumsum(rng.integers(0, 1 << 20, 5000).astype(np.uint64))[::-1]
    for eps in (3, 1000):
        for F in (0, 20):
            check_all(lc, high, eps, 8, rng, nq=200, frac_bits=F, fit="opt")
    low_high = np.concatenate([np.arange(0, 100, 3, dtype=np.uint64), high[-40:]])
    check_all(lc, low_high, 7, 6, rng, nq=100, fit="opt")


def test_opt_fit_large_hulls(lc):
    """Strictly convex keys (i^2) keep every key of a segment on the lower
    hull and pop the upper one back to two vertices at every key; concave
    keys (sqrt) the other way round.  With eps large enough for one segment
    per block, hulls reach 1024 vertices, so each step's scan takes 16 passes
    of the wave and the pops run long."""
    rng = np.random.default_rng(8)
    n = 6 * 1024 + 77
    i = np.arange(n, dtype=np.uint64)
    convex = i * i
    concave = np.floor(1e9 * np.sqrt(np.arange(n, dtype=np.float64))).astype(np.uint64)
    for keys in (convex, concave, convex.astype(np.uint32)):
        for eps, F in ((1 << 20, 0), (1 << 20, 20), (1 << 30, 0)):
            check_all(lc, keys, eps, 10, rng, nq=200, frac_bits=F, fit="opt")
    # segments of a few hundred keys inside blocks: hulls grow, the segment closes, they reset
    check_all(lc, convex, 1 << 12, 10, rng, nq=200, frac_bits=0, fit="opt")
    check_all(lc, concave, 1 << 16, 12, rng, nq=200, frac_bits=20, fit="opt")


@pytest.mark.parametrize("frac_bits", [0, 20, 32])
def test_opt_fit_short_and_long_segments_alternate(lc, frac_bits):
    rng = np.random.default_rng(95 + frac_bits)
    parts, pos = [], np.uint64(5)
    cap_gap = np.uint64(1) << np.uint64(64 - frac_bits) if frac_bits else np.uint64(0)
    for k in range(40):
        if k % 2 == 0:
            m, g = int(rng.integers(5, 400)), int(rng.integers(0, 50))
            run = pos + np.uint64(g) * np.arange(m, dtype=np.uint64)
        else:
            m = int(rng.integers(3, 300))
            gaps = rng.integers(1, 1 << 30, m).astype(np.uint64)
            if frac_bits and k % 6 == 1:
                gaps[rng.integers(0, m)] = cap_gap
            run = pos + np.cumsum(gaps, dtype=np.uint64)
        parts.append(run)
        pos = run[-1] + np.uint64(1)
        if pos > np.uint64(1) << np.uint64(62):
            break
    keys = np.concatenate(parts)
    for eps in (0, 3, 100):
        for log2b in (6, 10):
            check_all(lc, keys, eps, log2b, rng, nq=200, frac_bits=frac_bits, fit="opt")


def test_opt_fit_width_combinations(lc):
    rng = np.random.default_rng(20)
    for keys, eps, F in _width_combo_lists()[1::4]:
        check_all(lc, keys, eps, 6, rng, nq=32, frac_bits=F, fit="opt")


def _opt_frac4_lists():
    """Lists at F = 20 (4-byte fractions) for the optimal fit: the width
    lists, plus 64-key blocks of one or two flat runs and 1-key tail blocks,
    whose slopes take 1 or 2 bytes."""
    out = [(k, e, 20) for k, e, _ in _width_combo_lists()]
    rng = np.random.default_rng(5)
    for eps in (0, 1, 7, 255, 70000, (1 << 31) - 1):
        for jump in (1, 300, 1 << 20, 1 << 40):
            vals = np.cumsum(rng.integers(1, 3, 6)).astype(np.uint64) * np.uint64(jump)
            out.append((np.concatenate([np.repeat(vals, 64), vals[-1:] + np.uint64(jump)]), eps, 20))
            out.append((np.repeat(np.arange(12, dtype=np.uint64) * np.uint64(jump), 32), eps, 20))
    return out


def test_opt_fit_frac4_width_combinations(lc):
    """The block decoder has a loop per (anchor, slope) byte width for 4-byte
    fractions; every pair an optimal-fit blob reaches at F = 20 is decoded
    (lists chosen on the CPU by the pairs their oracle blobs use)."""
    rng = np.random.default_rng(21)
    seen = set()
    for keys, eps, F in _opt_frac4_lists():
        blob = oracle.compress(keys, eps, 6, F, fit="opt")
        h = oracle.header(blob)
        d = blob[h["off_dir"]:h["off_dir"] + 16 * h["nblocks"]].reshape(-1, 16)
        pairs = set(zip(d[:, 14].tolist(), d[:, 15].tolist()))
        if pairs <= seen:
            continue
        seen |= pairs
        check_all(lc, keys, eps, 6, rng, nq=64, frac_bits=F, fit="opt")
    want = {(a, s) for a in (1, 2, 4, 8) for s in (1, 2, 4, 8)} - {(8, 1)}
    assert want <= seen, sorted(want - seen)


def test_opt_fit_configs_reduced(lc, wl):
    """The benchmark recipes at sizes the oracle's optimal fit finishes in
    seconds, at F = 20 and F = 0."""
    rng = np.random.default_rng(4)
    keys = wl.as_numpy(wl.uniform_gaps(1_000_000, device="cpu"))
    for F in (0, 20):
        check_all(lc, keys, 31, 10, rng, nq=20_000, frac_bits=F, fit="opt")
    keys = wl.as_numpy(wl.lognormal_distinct(1_000_000, device="cpu"))
    for eps in (15, 255):
        check_all(lc, keys, eps, 10, rng, nq=20_000, fit="opt")
    keys = wl.as_numpy(wl.heterogeneous_runs(300_000, device="cpu", run_lo=1e3, run_hi=1e5))
    check_all(lc, keys, 63, 10, rng, nq=20_000, frac_bits=0, fit="opt")
    keys = wl.as_numpy(wl.lognormal_gaps(1_000_000, device="cpu"))
    check_all(lc, keys, 255, 10, rng, nq=20_000, fit="opt")


def test_opt_fit_determinism_and_unsorted(lc):
    rng = np.random.default_rng(3)
    keys = np.cumsum(rng.integers(0, 1000, 300_000)).astype(np.uint64)
    d = _to_dev(keys)
    assert torch.equal(lc.compress(d, 63, fit="opt").data, lc.compress(d, 63, fit="opt").data)
    m, o = lc.compress(d, 63, fit="min"), lc.compress(d, 63, fit="opt")
    assert o.info.nseg_total <= m.info.nseg_total and o.info.flags == 1 and m.info.flags == 0
    bad = keys[:5000].copy()
    bad[2500] = bad[2499] - np.uint64(1)
    with pytest.raises(lc.LcError):
        lc.compress(_to_dev(bad), 15, fit="opt")


# --- greedy fit with one block per lane: lists of at least 16384 blocks -------

LANES_MIN_BLOCKS = 16384  # lc_compress switches to the lane-per-block fit from here


def _big_keys(rng, n, kb, kind):
    """n sorted keys whose span fits the key width: small gaps, duplicates,
    wide gaps, or small gaps with rare jumps; shifted to the top of the range
    a third of the time."""
    wide = 12 if kb == 4 else 20
    if kind == "uniform":
        g = rng.integers(0, 100, n)
    elif kind == "dups":
        g = rng.integers(0, 2, n)
    elif kind == "wide":
        g = rng.integers(0, 1 << wide, n)
    else:
        g = rng.integers(0, 5, n)
        jumps = rng.random(n) < 0.01
        g[jumps] = rng.integers(1000, 1 << (wide + 6), int(jumps.sum()))
    k = np.cumsum(g.astype(np.uint64))
    hi = (1 << (8 * kb)) - 1
    assert int(k[-1]) <= hi
    base = hi - int(k[-1]) if rng.random() < 1 / 3 else 0
    return (k + np.uint64(base)).astype(np.uint32 if kb == 4 else np.uint64)


@pytest.mark.parametrize("kb", [4, 8])
def test_lanes_fit_random_lists(lc, kb):
    """16385 blocks of 64 keys (a partial last block, a block count that is
    not a multiple of 64) in four key shapes, eps / F pairs from exact to wide."""
    rng = np.random.default_rng(200 + kb)
    n = 64 * LANES_MIN_BLOCKS + 37
    for kind in ("uniform", "dups", "wide", "bursty"):
        keys = _big_keys(rng, n, kb, kind)
        for eps, F in ((0, 20), (3, 0), (63, 20), (4095, 32)):
            check_all(lc, keys, eps, 6, rng, nq=300, frac_bits=F)


@pytest.mark.parametrize("frac_bits", [0, 20, 32])
def test_lanes_fit_cap_gaps_and_runs(lc, frac_bits):
    """Arithmetic runs and sparse stretches with gaps at the overflow cap,
    repeated past 16384 blocks of 64 keys."""
    rng = np.random.default_rng(300 + frac_bits)
    parts, pos, total = [], np.uint64(5), 0
    cap_gap = np.uint64(1) << np.uint64(64 - frac_bits) if frac_bits else np.uint64(1) << np.uint64(40)
    k = 0
    while total < 64 * LANES_MIN_BLOCKS + 100:
        if k % 2 == 0:
            m, g = int(rng.integers(5, 2000)), int(rng.integers(0, 50))
            run = pos + np.uint64(g) * np.arange(m, dtype=np.uint64)
        else:
            m = int(rng.integers(3, 300))
            gaps = rng.integers(1, 1 << 20, m).astype(np.uint64)
            if k % 6 == 1 and pos < (np.uint64(1) << np.uint64(62)) - cap_gap:
                gaps[rng.integers(0, m)] = cap_gap
            run = pos + np.cumsum(gaps, dtype=np.uint64)
        parts.append(run)
        pos = run[-1] + np.uint64(1)
        total += m
        k += 1
        if pos > np.uint64(1) << np.uint64(62):
            pos = np.uint64(1) << np.uint64(62)
    keys = np.sort(np.concatenate(parts))[:64 * LANES_MIN_BLOCKS + 100]
    for eps in (0, 3, 100):
        check_all(lc, keys, eps, 6, rng, nq=300, frac_bits=frac_bits)


def test_lanes_fit_blocks_of_1024(lc, wl):
    """The benchmark's block size: 16.8M lognormal keys (16384 blocks plus a
    partial one), eps 63 and 255."""
    rng = np.random.default_rng(7)
    keys = wl.as_numpy(wl.lognormal_distinct(1024 * LANES_MIN_BLOCKS + 500, device="cpu"))
    for eps in (63, 255):
        check_all(lc, keys, eps, 10, rng, nq=20_000)


def test_lanes_fit_unsorted_and_determinism(lc):
    rng = np.random.default_rng(8)
    keys = np.cumsum(rng.integers(0, 100, 64 * LANES_MIN_BLOCKS + 64)).astype(np.uint64)
    d = _to_dev(keys)
    assert torch.equal(lc.compress(d, 15, 6).data, lc.compress(d, 15, 6).data)
    for pos in (64 * 5000, 64 * 5000 + 17, len(keys) - 1):  # at a block boundary, inside, last key
        bad = keys.copy()
        bad[pos] = bad[pos - 1] - np.uint64(1)
        with pytest.raises(lc.LcError):
            lc.compress(_to_dev(bad), 15, 6)


def test_corrupt_directory_entries_skip_their_blocks(lc):
    """Directory entries inconsistent with the layout (a segment area past the
    blob or before its region, no segments, an invalid byte width, a wrong
    key count) make the block decoders -- the full decode and ranges, with
    their staging workgroups -- skip those blocks and write nothing there;
    every other block decodes.  (Point queries: the next test.)"""
    rng = np.random.default_rng(21)
    keys = np.cumsum(rng.integers(1, 100, 40 * 1024 + 77)).astype(np.uint64)
    blob = lc.compress(_to_dev(keys), 63)
    h = blob.info
    data = blob.data.cpu().numpy().copy()
    dirs = data[h.off_dir:h.off_dir + 16 * h.nblocks].reshape(-1, 16)
    bad = {
        0: lambda d: d[0:8].view(np.uint64).__setitem__(0, h.blob_bytes + 4096),
        3: lambda d: d[0:8].view(np.uint64).__setitem__(0, h.off_seg - 16),
        11: lambda d: d[8:12].view(np.uint32).__setitem__(0, 0),
        20: lambda d: d.__setitem__(14, 3),
        33: lambda d: d[12:14].view(np.uint16).__setitem__(0, 5),
        40: lambda d: d[8:12].view(np.uint32).__setitem__(0, 0xFFFFFFFF),
    }
    for b, f in bad.items():
        row = dirs[b].copy()
        f(row)
        dirs[b] = row
    data[h.off_dir:h.off_dir + 16 * h.nblocks] = dirs.ravel()
    cb = lc.Blob.from_device(torch.from_numpy(data).to(DEV))
    n = len(keys)
    B = 1 << h.log2_block
    out = torch.full((n,), -1, dtype=torch.int64, device=DEV)
    lc.decompress(cb, out=out)
    got = out.cpu().numpy()
    for b in range(h.nblocks):
        lo, hi = b * B, min(n, (b + 1) * B)
        if b in bad:
            assert np.all(got[lo:hi] == -1), b
        else:
            assert np.array_equal(got[lo:hi].view(np.uint64), keys[lo:hi]), b
    for a, e in ((0, n), (5 * B + 7, 25 * B + 3), (10 * B, 12 * B), (39 * B + 1, n)):
        o = torch.full((e - a,), -1, dtype=torch.int64, device=DEV)
        lc.decompress_range(cb, a, e, out=o)
        g = o.cpu().numpy()
        for b in range(a // B, (e - 1) // B + 1):
            lo, hi = max(a, b * B), min(e, (b + 1) * B)
            if b in bad:
                assert np.all(g[lo - a:hi - a] == -1), (a, e, b)
            else:
                assert np.array_equal(g[lo - a:hi - a].view(np.uint64), keys[lo:hi]), (a, e, b)


def test_corrupt_directory_entries_in_point_queries(lc):
    """access and lower_bound check the directory entry they read: an
    index in a block with an inconsistent entry answers 0 and raises
    LC_FLAG_BADLIST (access), a query whose block is inconsistent answers n
    (lower_bound); every other query gives the definitions' answers."""
    rng = np.random.default_rng(22)
    keys = np.cumsum(rng.integers(1, 100, 40 * 1024 + 77)).astype(np.uint64)
    blob = lc.compress(_to_dev(keys), 63)
    h = blob.info
    data = blob.data.cpu().numpy().copy()
    dirs = data[h.off_dir:h.off_dir + 16 * h.nblocks].reshape(-1, 16)
    bad = {
        0: lambda d: d[0:8].view(np.uint64).__setitem__(0, h.blob_bytes + 4096),
        3: lambda d: d[0:8].view(np.uint64).__setitem__(0, h.off_seg - 16),
        11: lambda d: d[8:12].view(np.uint32).__setitem__(0, 0),
        20: lambda d: d.__setitem__(14, 3),
        33: lambda d: d[12:14].view(np.uint16).__setitem__(0, 5),
        40: lambda d: d[8:12].view(np.uint32).__setitem__(0, 0xFFFFFFFF),
    }
    for b, f in bad.items():
        row = dirs[b].copy()
        f(row)
        dirs[b] = row
    data[h.off_dir:h.off_dir + 16 * h.nblocks] = dirs.ravel()
    cb = lc.Blob.from_device(torch.from_numpy(data).to(DEV))
    n = len(keys)
    B = 1 << h.log2_block
    # access: every block's first, middle and last index
    idx = np.unique(np.concatenate([[b * B, b * B + B // 2, min(n, (b + 1) * B) - 1] for b in range(h.nblocks)]))
    idx = idx[idx < n]
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    got = lc.access(cb, torch.from_numpy(idx.astype(np.int64)).to(DEV), flags=flags, check=False).cpu().numpy()
    got = got.view(np.uint64)
    blk = idx // B
    in_bad = np.isin(blk, list(bad))
    assert np.all(got[in_bad] == 0)
    assert np.array_equal(got[~in_bad], keys[idx[~in_bad]])
    assert int(flags.item()) == lc.LC_FLAG_BADLIST
    # an intact blob raises no flag for the same indices
    flags.zero_()
    lc.access(blob, torch.from_numpy(idx.astype(np.int64)).to(DEV), flags=flags, check=False)
    assert int(flags.item()) == 0
    # lower_bound: keys, keys + 1 and keys - 1 in every block
    q = np.unique(np.concatenate([keys[idx], keys[idx] + np.uint64(1), keys[idx] - np.uint64(1)]))
    pos = lc.lower_bound(cb, torch.from_numpy(q.view(np.int64)).to(DEV)).cpu().numpy().astype(np.uint64)
    want = np.searchsorted(keys, q, side="left").astype(np.uint64)
    # the block a query searches: the last whose first key is < q
    first = keys[::B]
    qb = np.searchsorted(first, q, side="left").astype(np.int64) - 1
    hit = (qb >= 0) & np.isin(qb, list(bad))
    assert np.all(pos[hit] == n)
    assert np.array_equal(pos[~hit], want[~hit])
