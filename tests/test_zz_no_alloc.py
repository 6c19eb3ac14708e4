"""lc_compress_noalloc (the compress entry point whose workspace is the
library's static device scratch) against lc_compress with a caller
workspace, through the C ABI: byte-equal blobs, equal sizes and flags, on
calls in a row on one device where each later call is smaller than the one
before (the scratch keeps the previous call's contents), on every fit path
the scratch can hold: the 4-blocks-per-workgroup greedy fit, the
one-block-per-lane greedy fit (at 64-key blocks, where enough blocks fit in
the scratch), the fewest-segment fit and the optimal fit.  Blobs of the first
pair are also decoded back to the keys (Def. 1)."""
import sys

import numpy as np
import pytest
import torch

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


def _pair(lc, keys, eps, log2b=10, frac_bits=0, fit="greedy"):
    """(blob via lc_compress, blob via lc_compress_noalloc), each trimmed to
    its reported size; flags of both calls must stay 0."""
    n = keys.numel()
    kb = 4 if keys.dtype in (torch.int32, torch.uint32) else 8
    blob_max, ws_bytes = lc.compress_bound(n, kb, eps, log2b, frac_bits, fit)
    assert ws_bytes <= lc.NOALLOC_SCRATCH_BYTES, (n, ws_bytes)
    _say(f"noalloc case n={n} kb={kb} eps={eps} log2b={log2b} F={frac_bits} fit={fit} ws={ws_bytes}")
    out = []
    for noalloc in (False, True):
        blob = torch.full((blob_max,), 0xAB, dtype=torch.uint8, device=DEV)
        nbytes = torch.zeros(1, dtype=torch.int64, device=DEV)
        flags = torch.zeros(1, dtype=torch.int32, device=DEV)
        if noalloc:
            lc.compress_noalloc_async(keys, eps, blob, nbytes, flags, log2b, frac_bits, fit=fit)
        else:
            ws = torch.empty(max(ws_bytes, 16), dtype=torch.uint8, device=DEV)
            lc.compress_async(keys, eps, blob, ws, nbytes, flags, log2b, frac_bits, fit=fit)
        torch.cuda.synchronize()
        assert int(flags.item()) == 0, (noalloc, int(flags.item()))
        out.append(blob[:int(nbytes.item())].clone())
    return out


def test_noalloc_equals_compress_on_calls_in_a_row(lc, wl):
    # 1: 3e6 u64 keys with lognormal gaps, 1024-key blocks (workgroup fit);
    # 2: 2e6 u32 keys at 64-key blocks (31,250 blocks: the per-lane fit and
    #    the code-packing kernel); 3, 4: smaller inputs through the other fits
    cases = [
        (wl.lognormal_gaps(3_000_000, seed=wl.SEED_BASE + 900, device=DEV), 63, 10, 0, "greedy"),
        (wl.uniform_gaps(2_000_000, seed=wl.SEED_BASE + 901, device=DEV), 15, 6, 0, "greedy"),
        (wl.uniform_gaps(300_000, seed=wl.SEED_BASE + 902, device=DEV), 31, 10, 20, "min"),
        (wl.lognormal_gaps(100_000, seed=wl.SEED_BASE + 903, device=DEV), 63, 10, 0, "opt"),
        (wl.uniform_gaps(5_000, seed=wl.SEED_BASE + 904, device=DEV), 7, 10, 20, "greedy"),
    ]
    prev = None
    for i, (keys, eps, log2b, F, fit) in enumerate(cases):
        n = keys.numel()
        assert prev is None or n < prev
        prev = n
        ref, got = _pair(lc, keys, eps, log2b, F, fit)
        assert got.numel() == ref.numel(), (i, got.numel(), ref.numel())
        assert torch.equal(got, ref), f"case {i}: noalloc blob differs from lc_compress's"
        if i == 0:
            blob = lc.Blob(got, lc.info(got[:lc.HEADER_BYTES].cpu()))
            assert torch.equal(lc.decompress(blob), keys), "round trip of the noalloc blob (Def. 1)"


def test_noalloc_rejects_what_the_scratch_cannot_hold(lc):
    # the largest n whose workspace fits, and one block more: LC_ETOOBIG,
    # raised on the host before anything is enqueued
    B = 1 << 10
    lo, hi = 1, 1 << 30
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if lc.compress_bound(mid, 8, 63, 10, 0)[1] <= lc.NOALLOC_SCRATCH_BYTES:
            lo = mid
        else:
            hi = mid - 1
    n_max = lo
    assert n_max > 3_500_000 and n_max % B == 0
    keys = torch.arange(n_max + 1, dtype=torch.int64, device=DEV)
    blob = torch.empty(lc.compress_bound(n_max + 1, 8, 63, 10, 0)[0], dtype=torch.uint8, device=DEV)
    nbytes = torch.zeros(1, dtype=torch.int64, device=DEV)
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    with pytest.raises(lc.LcError) as ei:
        lc.compress_noalloc_async(keys, 63, blob, nbytes, flags, 10, 0)
    assert "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert int(nbytes.item()) == 0 and int(flags.item()) == 0
    # and n_max itself is accepted and equals lc_compress
    ref, got = _pair(lc, keys[:n_max], 63, 10, 0)
    assert torch.equal(got, ref)
