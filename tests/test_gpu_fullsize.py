"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (blocks of 1024 keys, F = 20).

The oracle cannot encode 1e8 keys in a test's time, so these checks use:
  * properties that hold at any size -- decode(compress(K)) == K exactly
    (Def. 1), directory offsets equal to the prefix sums of the per-block
    segment areas, and the blob size equal to its closed form;
  * sampled outputs the oracle computes one by one -- a block's bytes depend
    only on its keys, so the oracle compresses each sampled block on its own
    and its slab, segment area and directory fields must equal the GPU
    blob's;
  * sampled queries against the plain definitions (K[i], K[b:e],
    searchsorted(K, q, 'left')).
"""
import sys

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def a16(x):
    return (x + 15) // 16 * 16


def check_fullsize(lc, keys: torch.Tensor, eps: int, n_access: int, n_lb: int, seed: int, fit: str = "greedy",
                   frac_bits: int = 20):
    n = keys.numel()
    kb = keys.element_size()
    _say(f"full-size case n={n} kb={kb} eps={eps} fit={fit} F={frac_bits}")
    blob = lc.compress(keys, eps, 10, frac_bits, fit=fit)  # log2_block 10 as the benchmark
    h = blob.info
    B = 1 << h.log2_block
    assert h.n == n and h.nblocks == (n + B - 1) // B

    out = lc.decompress(blob)
    assert torch.equal(out, keys), "round trip (Def. 1)"
    del out

    data = blob.data.cpu().numpy()
    dirs = data[h.off_dir:h.off_dir + 16 * h.nblocks].reshape(-1, 16)
    seg_off = dirs[:, 0:8].copy().view(np.uint64).ravel().astype(np.int64)
    nseg = dirs[:, 8:12].copy().view(np.uint32).ravel().astype(np.int64)
    nk = dirs[:, 12:14].copy().view(np.uint16).ravel().astype(np.int64) + 1
    ab = dirs[:, 14].astype(np.int64)
    sb = dirs[:, 15].astype(np.int64)
    fb = 0 if not h.flags or frac_bits == 0 else 1 if frac_bits <= 8 else 2 if frac_bits <= 16 else 4
    area = a16(2 * nseg) + a16(ab * nseg) + a16(sb * nseg) + a16(fb * nseg)
    assert np.array_equal(seg_off, h.off_seg + np.concatenate([[0], np.cumsum(area)[:-1]]))
    assert h.blob_bytes == h.off_seg + int(area.sum()) == len(data)
    assert h.nseg_total == int(nseg.sum()) and h.max_nseg == int(nseg.max())
    assert h.max_seg_bytes == int(area.max())
    assert np.all(nk[:-1] == B) and nk[-1] == n - (h.nblocks - 1) * B

    rng = np.random.default_rng(seed)
    host = keys.cpu().numpy().view(np.uint32 if kb == 4 else np.uint64)
    picks = set(rng.choice(h.nblocks, size=min(48, h.nblocks), replace=False).tolist())
    picks |= {0, h.nblocks - 1, int(np.argmax(nseg)), int(np.argmax(area))}
    for b in sorted(picks):
        kk = host[b * B:(b + 1) * B]
        one = oracle.compress(kk, eps, h.log2_block, frac_bits, fit=fit)
        oh = oracle.header(one)
        od = one[oh["off_dir"]:oh["off_dir"] + 16]
        assert np.array_equal(od[8:16], dirs[b, 8:16]), b
        assert np.array_equal(one[oh["off_res"]:oh["off_res"] + h.res_stride],
                              data[h.off_res + b * h.res_stride:h.off_res + (b + 1) * h.res_stride]), b
        assert np.array_equal(one[oh["off_seg"]:oh["blob_bytes"]], data[seg_off[b]:seg_off[b] + area[b]]), b
        assert int.from_bytes(bytes(data[h.off_first + b * kb:h.off_first + (b + 1) * kb]), "little") == int(kk[0])

    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    idx = torch.randint(0, n, (n_access,), device=DEV, generator=g)
    assert torch.equal(lc.access(blob, idx), keys[idx])
    lo, hi = int(host[0]), int(host[-1])
    q = torch.randint(lo, hi + 2, (n_lb,), device=DEV, generator=g, dtype=torch.int64).to(keys.dtype)
    want = torch.searchsorted(keys, q, side="left")
    assert torch.equal(lc.lower_bound(blob, q), want)
    for _ in range(4):
        a = int(rng.integers(0, n))
        e = int(min(n, a + rng.integers(1, 5_000_000)))
        assert torch.equal(lc.decompress_range(blob, a, e), keys[a:e]), (a, e)
    assert torch.equal(lc.decompress_range(blob, n // 4, n // 4 + n // 2), keys[n // 4:n // 4 + n // 2])
    return blob


@pytest.fixture(scope="module")
def lc():
    from paper_2412_10770_amd import lc as mod
    return mod


@pytest.fixture(scope="module")
def wl():
    from paper_2412_10770_amd import workloads
    return workloads


# F = 0 is the benchmark's configuration, F = 20 the library default
@pytest.mark.parametrize("frac_bits", [0, 20])
def test_lognormal_100m(lc, wl, frac_bits):
    """100M distinct uint64 keys, lognormal(0, 2) scaled to 2^40; eps 15 / 63 / 255."""
    keys = wl.lognormal_distinct(100_000_000, device=DEV)
    for eps in (15, 63, 255):
        check_fullsize(lc, keys, eps, n_access=1_000_000, n_lb=1_000_000, seed=eps, frac_bits=frac_bits)


def test_lognormal_100m_min_fit(lc, wl):
    """The fewest-segment fit on the same 100M keys: never more segments than
    the greedy fit, same checks."""
    keys = wl.lognormal_distinct(100_000_000, device=DEV)
    for eps in (63, 255):
        g = lc.compress(keys, eps, frac_bits=20).info.nseg_total
        m = check_fullsize(lc, keys, eps, n_access=1_000_000, n_lb=1_000_000, seed=100 + eps, fit="min")
        assert m.info.nseg_total <= g


def test_lognormal_100m_opt_fit(lc, wl):
    """The optimal fit (free fixed-point intercepts) on the same 100M keys, at
    F = 20 (4-byte fractions) and F = 0 (none): never more segments than the
    fewest-segment anchored fit at F = 20, same checks."""
    keys = wl.lognormal_distinct(100_000_000, device=DEV)
    m = lc.compress(keys, 63, frac_bits=20, fit="min").info.nseg_total
    for F in (20, 0):
        o = check_fullsize(lc, keys, 63, n_access=1_000_000, n_lb=1_000_000, seed=300 + F, fit="opt", frac_bits=F)
        assert o.info.flags == 1
        if F == 20:
            assert o.info.nseg_total <= m


def test_heterogeneous_runs_200m_opt_fit(lc, wl):
    """Dense runs: segments span whole blocks, so the hulls grow long."""
    keys = wl.heterogeneous_runs(200_000_000, device=DEV)
    check_fullsize(lc, keys, 63, n_access=1_000_000, n_lb=1_000_000, seed=5, fit="opt", frac_bits=0)


def test_heterogeneous_runs_200m_min_fit(lc, wl):
    """Dense runs: every anchor's cone stays open across much of its block."""
    keys = wl.heterogeneous_runs(200_000_000, device=DEV)
    check_fullsize(lc, keys, 63, n_access=1_000_000, n_lb=1_000_000, seed=4, fit="min")


@pytest.mark.parametrize("frac_bits", [0, 20])
def test_heterogeneous_runs_200m(lc, wl, frac_bits):
    """200M uint64 keys, alternating dense / Zipf(1.2) runs; eps 63; 10M access, 1M lower_bound."""
    keys = wl.heterogeneous_runs(200_000_000, device=DEV)
    check_fullsize(lc, keys, 63, n_access=10_000_000, n_lb=1_000_000, seed=3, frac_bits=frac_bits)


@pytest.mark.parametrize("frac_bits", [0, 20])
def test_posting_lists_4096(lc, wl, frac_bits):
    """The batch workload at full size: 4096 uint32 lists (~2.9e8 keys), eps
    autotuned over {7, 31, 127}.  Whole-batch round trip; on sampled lists
    (the longest, the shortest and random ones) the chosen eps equals the
    argmin of the oracle's exact sizes and the blob equals the oracle's."""
    cands = (7, 31, 127)
    keys, lengths = wl.posting_lists(4096, device=DEV)
    _say(f"posting lists full size: {keys.numel()} keys, F={frac_bits}")
    batch = lc.batch_compress(keys, lengths, candidates=cands, frac_bits=frac_bits)
    assert torch.equal(lc.batch_decompress(batch), keys)
    host = keys.cpu().numpy().view(np.uint32)
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]])
    rng = np.random.default_rng(4096)
    picks = set(rng.choice(len(lengths), 16, replace=False).tolist())
    picks |= {int(np.argmax(lengths)), int(np.argmin(lengths))}
    for l in sorted(picks):
        x = host[offs[l]:offs[l] + lengths[l]]
        blobs = [oracle.compress(x, e, 10, frac_bits) for e in cands]
        best = int(np.argmin([len(b) for b in blobs]))
        assert batch.eps[l] == cands[best], l
        assert np.array_equal(batch.blob(l).data.cpu().numpy(), blobs[best]), l


def check_sampled_blocks(lc, blob, keys: torch.Tensor, eps: int, frac_bits: int, seed: int, count: int = 48):
    """Blocks sampled from a blob too large to copy whole: the first, the
    last, the one with the most segments and `count` random ones, each
    compared byte for byte with the oracle's blob of that block alone
    (directory fields, residual slab, segment area, first key), reading only
    the directory and the sampled blocks' bytes from the device."""
    h = blob.info
    B = 1 << h.log2_block
    kb = keys.element_size()
    d = blob.data
    dirs = d[h.off_dir:h.off_dir + 16 * h.nblocks].cpu().numpy().reshape(-1, 16)
    seg_off = dirs[:, 0:8].copy().view(np.uint64).ravel().astype(np.int64)
    nseg = dirs[:, 8:12].copy().view(np.uint32).ravel().astype(np.int64)
    ab = dirs[:, 14].astype(np.int64)
    sb = dirs[:, 15].astype(np.int64)
    area = a16(2 * nseg) + a16(ab * nseg) + a16(sb * nseg)
    assert np.array_equal(seg_off, h.off_seg + np.concatenate([[0], np.cumsum(area)[:-1]]))
    assert h.blob_bytes == h.off_seg + int(area.sum())
    rng = np.random.default_rng(seed)
    picks = set(rng.choice(h.nblocks, size=min(count, h.nblocks), replace=False).tolist())
    picks |= {0, h.nblocks - 1, int(np.argmax(nseg))}
    dt = np.uint32 if kb == 4 else np.uint64
    for b in sorted(picks):
        kk = keys[b * B:(b + 1) * B].cpu().numpy().view(dt)
        one = oracle.compress(kk, eps, h.log2_block, frac_bits)
        oh = oracle.header(one)
        assert np.array_equal(one[oh["off_dir"] + 8:oh["off_dir"] + 16], dirs[b, 8:16]), b
        slab = d[h.off_res + b * h.res_stride:h.off_res + (b + 1) * h.res_stride].cpu().numpy()
        assert np.array_equal(one[oh["off_res"]:oh["off_res"] + h.res_stride], slab), b
        seg = d[int(seg_off[b]):int(seg_off[b] + area[b])].cpu().numpy()
        assert np.array_equal(one[oh["off_seg"]:oh["blob_bytes"]], seg), b
        fk = d[h.off_first + b * kb:h.off_first + (b + 1) * kb].cpu().numpy()
        assert int.from_bytes(bytes(fk), "little") == int(kk[0]), b
    return len(picks)


def test_serving_store_1e9(lc, wl):
    """The serving workload at full size: 1e9 uint64 keys with lognormal
    gaps, stored at the eps with the smallest blob among {15, 63, 255, 1023}
    (checked against all four sizes); ~50 blocks of the stored blob equal
    the oracle's (check_sampled_blocks); the whole store decodes back to the
    keys, slice by slice (Def. 1); 3000 mixed Poisson requests served with
    results copied out and compared with the definitions computed by torch
    from the raw keys on the device (K[a:b], K[i], searchsorted).  F = 0,
    as the benchmark."""
    n = 1_000_000_000
    keys = wl.lognormal_gaps(n, seed=wl.SEED_BASE + 5, device=DEV)
    _say("serving store 1e9")
    sizes = {}
    for e in (15, 63, 255, 1023):
        b = lc.compress(keys, e, frac_bits=0)
        sizes[e] = b.nbytes
        del b
        torch.cuda.empty_cache()
    eps = min(sizes, key=lambda e: (sizes[e], e))
    blob = lc.compress(keys, eps, frac_bits=0)
    assert blob.nbytes == sizes[eps]
    _say(f"serving store 1e9: eps {eps}, sampled blocks against the oracle")
    assert check_sampled_blocks(lc, blob, keys, eps, 0, seed=1009) >= 48
    _say("serving store 1e9: sliced round trip")
    step = 125_000_000
    for a in range(0, n, step):
        e = min(n, a + step)
        assert torch.equal(lc.decompress_range(blob, a, e), keys[a:e]), (a, e)
    torch.cuda.empty_cache()
    lo, hi = int(keys[0]), int(keys[-1])
    op, a, b, arr = wl.request_stream(3000, n, lo, hi, 1e6, seed=77)
    size = np.where(op == 1, (b - a) * 8, 8).astype(np.int64)
    off = np.concatenate([[0], np.cumsum((size + 15) // 16 * 16)[:-1]]).astype(np.int64)
    buf = torch.zeros(int(off[-1] + size[-1] + 16), dtype=torch.uint8, device=DEV)
    with lc.Server(blob) as srv:
        res, st = srv.run(lc.requests(op, a, b, arr, buf.data_ptr() + off))
    torch.cuda.synchronize()
    assert np.all(res["status"] == 0) and st["launches"] >= 1
    i64 = torch.int64
    for i in range(len(op)):
        seg = buf[int(off[i]):int(off[i] + size[i])].view(i64)
        if op[i] == 1:
            assert torch.equal(seg, keys[int(a[i]):int(b[i])]), ("range", i)
        elif op[i] == 2:
            assert int(seg[0]) == int(keys[int(a[i])]), ("access", i)
        else:
            q = torch.tensor([int(a[i])], dtype=i64, device=DEV)
            assert int(seg[0]) == int(torch.searchsorted(keys, q, side="left")[0]), ("lower_bound", i)


def test_grid_chunking_past_2_22_workgroups(lc, wl):
    """1.1e9 uint32 keys in 64-key blocks: more than 2^22 fit workgroups
    (four blocks each) and decode workgroups, so every launcher splits its
    grid into several launches.  Round trip, directory / size closed forms,
    blocks sampled on both sides of each split against the oracle, ranges
    across the splits, access and lower_bound samples."""
    n = 1_100_000_000
    g = torch.Generator(device=DEV)
    g.manual_seed(wl.SEED_BASE + 60)
    keys = torch.cumsum(torch.randint(0, 4, (n,), device=DEV, generator=g, dtype=torch.int32), 0,
                        dtype=torch.int64).to(torch.int32)  # gaps 0..3: < 2^32 in all
    _say("grid chunking: 1.1e9 u32 keys, 64-key blocks")
    blob = lc.compress(keys, 7, 6)
    h = blob.info
    assert h.nblocks > (1 << 22) * 4 and h.nblocks == (n + 63) // 64
    out = lc.decompress(blob)
    assert torch.equal(out, keys), "round trip (Def. 1)"
    del out
    data = blob.data.cpu().numpy()
    dirs = data[h.off_dir:h.off_dir + 16 * h.nblocks].reshape(-1, 16)
    seg_off = dirs[:, 0:8].copy().view(np.uint64).ravel().astype(np.int64)
    nseg = dirs[:, 8:12].copy().view(np.uint32).ravel().astype(np.int64)
    ab = dirs[:, 14].astype(np.int64)
    sb = dirs[:, 15].astype(np.int64)
    area = a16(2 * nseg) + a16(ab * nseg) + a16(sb * nseg)
    assert np.array_equal(seg_off[1:], seg_off[:-1] + area[:-1]) and seg_off[0] == h.off_seg
    assert h.blob_bytes == h.off_seg + int(area.sum()) == len(data)
    split_fit, split_dec = (1 << 22) * 4, 1 << 22  # first block of the second launch of each
    picks = {0, split_dec - 1, split_dec, split_dec + 1, 2 * split_dec, split_fit - 1, split_fit, split_fit + 3,
             h.nblocks - 1}
    for b in sorted(p for p in picks if p < h.nblocks):
        kk = keys[b * 64:(b + 1) * 64].cpu().numpy().view(np.uint32)
        one = oracle.compress(kk, 7, 6)
        oh = oracle.header(one)
        assert np.array_equal(one[oh["off_dir"] + 8:oh["off_dir"] + 16], dirs[b, 8:16]), b
        assert np.array_equal(one[oh["off_res"]:oh["off_res"] + h.res_stride],
                              data[h.off_res + b * h.res_stride:h.off_res + (b + 1) * h.res_stride]), b
        assert np.array_equal(one[oh["off_seg"]:oh["blob_bytes"]], data[seg_off[b]:seg_off[b] + area[b]]), b
    for a_, e_ in ((split_dec * 64 - 100, split_dec * 64 + 100), (split_fit * 64 - 5, split_fit * 64 + 77)):
        assert torch.equal(lc.decompress_range(blob, a_, e_), keys[a_:e_]), (a_, e_)
    idx = torch.randint(0, n, (100_000,), device=DEV, generator=g)
    assert torch.equal(lc.access(blob, idx), keys[idx])
    q = keys[idx[:10_000]] + 1  # uint32 bit patterns (wraps like the unsigned key)
    u = lambda t: t.to(torch.int64) & 0xFFFFFFFF  # noqa: E731
    want = torch.searchsorted(u(keys), u(q), side="left")
    assert torch.equal(lc.lower_bound(blob, q), want)
