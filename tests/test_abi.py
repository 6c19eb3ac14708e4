"""The C ABI library loads and exports what include/lc.h declares; host-side
argument checks (no GPU needed: every call here fails before any enqueue)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lc.h")).read()
    return sorted(set(re.findall(r"^(?:lc_status|const char\*)\s+(lc_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lc():
    from paper_2412_10770_amd import lc as mod
    return mod


def test_header_declares_the_five_operations():
    names = _declared()
    for op in ("lc_compress", "lc_decompress", "lc_decompress_range", "lc_access", "lc_lower_bound"):
        assert op in names


def test_library_exports_every_declared_symbol(lc):
    raw = ctypes.CDLL(lc.LIB_PATH)
    for name in _declared():
        assert hasattr(raw, name), name
    assert sorted(lc.EXPORTED) == _declared()


def test_strerror(lc):
    assert lc.strerror(0) == "ok"
    for code in (-1, -2, -3, -4, -5):
        assert lc.strerror(code) not in ("", "unknown status")


def test_noalloc_checks_on_the_host(lc):
    """lc_compress_noalloc refuses, before any device call, inputs whose
    workspace exceeds its static scratch (LC_ETOOBIG) and bad parameters."""
    p = lc.params(8, 63, 10, 0)
    assert lc.lib.lc_compress_noalloc(None, 10 ** 8, ctypes.byref(p), None, 0, None, None, None) == lc.LC_ETOOBIG
    assert lc.compress_bound(10 ** 8, 8, 63, 10, 0)[1] > lc.NOALLOC_SCRATCH_BYTES
    bad = lc.lc_params(3, 10, 0, 0, 63)
    assert lc.lib.lc_compress_noalloc(None, 10, ctypes.byref(bad), None, 0, None, None, None) == lc.LC_EINVAL
    assert lc.lib.lc_compress_noalloc(None, 2 ** 41, ctypes.byref(p), None, 0, None, None, None) == lc.LC_EINVAL


def test_compress_bound(lc):
    for n, kb, eps, log2b in ((0, 4, 0, 6), (1, 8, 63, 10), (10 ** 8, 8, 255, 10), (1000, 4, 7, 12)):
        blob_max, ws = lc.compress_bound(n, kb, eps, log2b)
        B = 1 << log2b
        nblocks = -(-n // B)
        w = int(np.ceil(np.log2(2 * eps + 1)))
        stride = -(-(-(-B * w // 8)) // 16) * 16
        fixed = 128 + -(-nblocks * kb // 16) * 16 + 16 * nblocks + nblocks * stride
        assert blob_max >= fixed + nblocks * 48
        assert ws >= 18 * nblocks * B
    for bad in ((3, 10, 20, 0), (8, 5, 20, 0), (8, 13, 20, 0), (8, 10, 33, 0), (8, 10, 20, 2 ** 31)):
        p = lc.lc_params(bad[0], bad[1], bad[2], 0, bad[3])
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        assert lc.lib.lc_compress_bound(10, ctypes.byref(p), ctypes.byref(a), ctypes.byref(b)) == lc.LC_EINVAL
    p = lc.params(8, 63)
    assert lc.lib.lc_compress_bound(2 ** 41, ctypes.byref(p), None, None) == lc.LC_EINVAL
    # the fit field: greedy (0) and fewest segments (1) share sizes; the
    # optimal fit (2) adds the intercept fractions (LC_FRAC_BYTES(F) per
    # segment, and 4 bytes per key slot of workspace); anything else is rejected
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    assert lc.lib.lc_compress_bound(5000, ctypes.byref(lc.params(8, 63, fit="min")), ctypes.byref(a), ctypes.byref(b)) == 0
    assert (a.value, b.value) == lc.compress_bound(5000, 8, 63)
    g_blob, g_ws = lc.compress_bound(5000, 8, 63)
    nblocks = -(-5000 // 1024)
    for F, fb in ((0, 0), (8, 1), (16, 2), (20, 4), (32, 4)):
        o_blob, o_ws = lc.compress_bound(5000, 8, 63, 10, F, fit="opt")
        assert o_blob == lc.compress_bound(5000, 8, 63, 10, F)[0] + nblocks * fb * 1024
        assert o_ws == g_ws + 4 * nblocks * 1024
    for fit in (3, 255):
        p = lc.lc_params(8, 10, 20, fit, 63)
        assert lc.lib.lc_compress_bound(10, ctypes.byref(p), None, None) == lc.LC_EINVAL
    with pytest.raises(ValueError):
        lc.params(8, 63, fit="optimal")
    assert lc.FITS["opt"] == 2


def test_info_parses_oracle_headers(lc):
    rng = np.random.default_rng(3)
    for kb, eps, log2b, n in ((4, 63, 10, 5000), (8, 0, 6, 1), (8, 4095, 12, 9000), (4, 7, 8, 0)):
        keys = np.cumsum(rng.integers(0, 50, n)).astype(np.uint32 if kb == 4 else np.uint64)
        for fit, F in (("greedy", 20), ("opt", 20), ("opt", 0), ("opt", 12)):
            blob = oracle.compress(keys, eps, log2b, F, fit=fit)
            inf = lc.info(blob[:128])
            h = oracle.header(blob)
            assert h["flags"] == (fit == "opt")
            for f in oracle.HEADER_FIELDS:
                assert getattr(inf, f) == h[f], (fit, F, f)


def test_info_rejects_bad_headers(lc):
    blob = oracle.compress(np.arange(0, 3000, 2, dtype=np.uint64), 15, 9)
    for off, val in ((0, 0), (4, 9), (6, 3), (7, 5), (9, 1), (10, 2), (11, 1), (24, 7), (56, 1)):
        bad = blob[:128].copy()
        bad[off] = val
        with pytest.raises(lc.LcError) as e:
            lc.info(bad)
        assert e.value.code == lc.LC_EFORMAT, off
    with pytest.raises(lc.LcError):
        lc.info(blob[:64])


def test_entry_points_reject_bad_arguments_before_any_launch(lc):
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails its checks first
    p = lc.params(8, 63)
    assert lc.lib.lc_compress(fake, 10, None, fake, 1 << 20, fake, 1 << 20, null, fake, null) == lc.LC_EINVAL
    assert lc.lib.lc_compress(fake, 10, ctypes.byref(p), null, 1 << 20, fake, 1 << 20, null, fake, null) == lc.LC_EINVAL
    assert lc.lib.lc_compress(fake, 10, ctypes.byref(p), fake, 1 << 20, fake, 1 << 20, null, null, null) == lc.LC_EINVAL
    assert lc.lib.lc_compress(fake, 10, ctypes.byref(p), fake, 16, fake, 1 << 20, null, fake, null) == lc.LC_ENOSPC
    assert lc.lib.lc_compress(fake, 10, ctypes.byref(p), fake, 1 << 20, fake, 16, null, fake, null) == lc.LC_ENOSPC
    assert lc.lib.lc_compress(ctypes.c_void_p(0x1001), 10, ctypes.byref(p), fake, 1 << 20, fake, 1 << 20, null,
                              fake, null) == lc.LC_EINVAL
    blob = oracle.compress(np.arange(0, 30000, 3, dtype=np.uint64), 63, 10)
    inf = lc.info(blob[:128])
    assert lc.lib.lc_decompress_range(fake, ctypes.byref(inf), 5, 4, fake, null) == lc.LC_EINVAL
    assert lc.lib.lc_decompress_range(fake, ctypes.byref(inf), 0, inf.n + 1, fake, null) == lc.LC_EINVAL
    assert lc.lib.lc_decompress_range(fake, ctypes.byref(inf), 7, 7, fake, null) == lc.LC_OK  # empty: no-op
    assert lc.lib.lc_decompress(fake, ctypes.byref(inf), ctypes.c_void_p(0x1004), null) == lc.LC_EINVAL
    assert lc.lib.lc_access(fake, ctypes.byref(inf), fake, 5, fake, null, null) == lc.LC_EINVAL
    assert lc.lib.lc_access(fake, ctypes.byref(inf), fake, 0, fake, null, null) == lc.LC_OK
    assert lc.lib.lc_lower_bound(null, ctypes.byref(inf), fake, 5, fake, null) == lc.LC_EINVAL
    inf.off_seg += 16  # info no longer consistent with the layout rules
    assert lc.lib.lc_decompress(fake, ctypes.byref(inf), fake, null) == lc.LC_EINVAL


def test_batch_plan(lc):
    """lc_batch_plan is host code: slots, block and group offsets, totals."""
    lengths = [0, 5, 1024, 1025, 100_000, 0, 64]
    for kb, log2b in ((4, 10), (8, 6), (4, 12)):
        p, t = lc.batch_plan(lengths, 7, kb, max_eps=127, log2_block=log2b)
        B = 1 << log2b
        nb = np.array([-(-n // B) for n in lengths])
        assert list(t["key_off"]) == list(np.concatenate([[0], np.cumsum(lengths)[:-1]]))
        assert list(t["block_off"]) == list(np.concatenate([[0], np.cumsum(nb)[:-1]]))
        ng = (nb + 3) // 4
        assert list(t["group_off"]) == list(np.concatenate([[0], np.cumsum(ng)[:-1]]))
        caps = [lc.compress_bound(n, kb, 127, log2b)[0] for n in lengths]
        assert list(t["blob_cap"]) == caps
        assert list(t["blob_off"]) == list(np.concatenate([[0], np.cumsum(caps)[:-1]]))
        assert all(int(o) % 16 == 0 for o in t["blob_off"])
        assert p.total_blocks == nb.sum() and p.total_groups == ng.sum() and p.blob_bytes == sum(caps)
        assert p.ws_bytes >= 18 * p.total_blocks * B + 8 * 16 * p.total_blocks
        assert list(t["eps"]) == [7] * len(lengths)
    # the optimal fit's slots hold the intercept fractions, its workspace one
    # u32 fraction per key slot more
    for F in (0, 20):
        g, _ = lc.batch_plan(lengths, 7, 8, max_eps=127, frac_bits=F)
        o, t = lc.batch_plan(lengths, 7, 8, max_eps=127, frac_bits=F, fit="opt")
        assert o.fit == 2 and g.fit == 0
        assert list(t["blob_cap"]) == [lc.compress_bound(n, 8, 127, 10, F, fit="opt")[0] for n in lengths]
        assert o.ws_bytes == g.ws_bytes + 4 * o.total_blocks * 1024
        m, t = lc.batch_plan(lengths, 7, 8, max_eps=127, frac_bits=F, fit="min")
        assert m.blob_bytes == g.blob_bytes and m.ws_bytes == g.ws_bytes


def test_batch_bad_args(lc):
    """Batch entry points reject bad parameters before any launch."""
    P = ctypes.byref
    t = np.zeros(2, dtype=lc.BATCH_LIST_DTYPE)
    t["n"] = [10, 20]
    good = lc.lc_batch_params(4, 10, 20, 0, 2, 31, 0, 0, 0, 0, 0)
    tp = t.ctypes.data_as(ctypes.c_void_p)
    for bad in (lc.lc_batch_params(3, 10, 20, 0, 2, 31, 0, 0, 0, 0, 0),
                lc.lc_batch_params(4, 5, 20, 0, 2, 31, 0, 0, 0, 0, 0),
                lc.lc_batch_params(4, 10, 33, 0, 2, 31, 0, 0, 0, 0, 0),
                lc.lc_batch_params(4, 10, 20, 0, 0, 31, 0, 0, 0, 0, 0),
                lc.lc_batch_params(4, 10, 20, 0, 2, 2 ** 31, 0, 0, 0, 0, 0),
                lc.lc_batch_params(4, 10, 20, 3, 2, 31, 0, 0, 0, 0, 0),  # no such tiling
                lc.lc_batch_params(4, 10, 20, 0, 2, 31, 3, 0, 0, 0, 0)):  # no such fit
        assert lc.lib.lc_batch_plan(P(bad), tp) == lc.LC_EINVAL
    assert lc.lib.lc_batch_plan(P(good), None) == lc.LC_EINVAL
    assert lc.lib.lc_batch_plan(P(good), tp) == lc.LC_OK
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every call below fails its checks first
    cands = (ctypes.c_uint32 * 3)(7, 31, 127)
    # null table / stats
    assert lc.lib.lc_batch_compress(fake, 30, None, P(good), fake, 1 << 30, fake, 1 << 30, fake, fake, None) == lc.LC_EINVAL
    assert lc.lib.lc_batch_compress(fake, 30, fake, P(good), fake, 1 << 30, fake, 1 << 30, fake, None, None) == lc.LC_EINVAL
    # buffers too small
    assert lc.lib.lc_batch_compress(fake, 30, fake, P(good), fake, good.blob_bytes - 16, fake, 1 << 30, fake, fake,
                                    None) == lc.LC_ENOSPC
    assert lc.lib.lc_batch_compress(fake, 30, fake, P(good), fake, 1 << 30, fake, good.ws_bytes - 16, fake, fake,
                                    None) == lc.LC_ENOSPC
    # misaligned blob
    assert lc.lib.lc_batch_compress(fake, 30, fake, P(good), ctypes.c_void_p((1 << 20) + 8), 1 << 30, fake, 1 << 30,
                                    fake, fake, None) == lc.LC_EINVAL
    # candidates: above max_eps, not increasing, too many, none
    for cs in ((7, 31, 127), (31, 7), tuple(range(9)), ()):
        arr = (ctypes.c_uint32 * max(1, len(cs)))(*cs)
        assert lc.lib.lc_batch_sizes(fake, 30, fake, P(good), arr, len(cs), fake, 1 << 30, fake, fake,
                                     None) == lc.LC_EINVAL
        assert lc.lib.lc_batch_pick_eps(fake, P(good), fake, arr, len(cs), None) == lc.LC_EINVAL
    assert lc.lib.lc_batch_sizes(fake, 30, fake, P(good), cands, 3, fake, 1 << 30, None, fake, None) == lc.LC_EINVAL
    # decompress: misaligned output, null table
    assert lc.lib.lc_batch_decompress(fake, 1 << 30, fake, P(good), 4096, ctypes.c_void_p((1 << 20) + 2), 30, fake,
                                      None) == lc.LC_EINVAL
    assert lc.lib.lc_batch_decompress(fake, 1 << 30, None, P(good), 4096, fake, 30, fake, None) == lc.LC_EINVAL


def test_setop_bound_and_bad_args(lc):
    """lc_setop_bound is host code: AND capacity min(n_a, n_b), OR n_a + n_b;
    key widths must match; bad arguments fail before any launch."""
    a = lc.info(oracle.compress(np.arange(0, 30000, 3, dtype=np.uint64), 63, 10)[:128])
    b = lc.info(oracle.compress(np.arange(0, 3000, 7, dtype=np.uint64), 15, 10)[:128])
    c32 = lc.info(oracle.compress(np.arange(0, 500, dtype=np.uint32), 7, 10)[:128])
    P = ctypes.byref
    om, ws = ctypes.c_uint64(), ctypes.c_uint64()
    assert lc.lib.lc_setop_bound(P(a), P(b), lc.SETOP_INTERSECT, P(om), P(ws)) == lc.LC_OK
    assert om.value == min(a.n, b.n) and ws.value >= min(a.n, b.n) * 9
    assert lc.lib.lc_setop_bound(P(a), P(b), lc.SETOP_UNION, P(om), P(ws)) == lc.LC_OK
    assert om.value == a.n + b.n and ws.value >= (a.n + b.n) * 17
    assert lc.lib.lc_setop_bound(P(a), P(c32), lc.SETOP_UNION, P(om), P(ws)) == lc.LC_EINVAL
    assert lc.lib.lc_setop_bound(P(a), P(b), 3, P(om), P(ws)) == lc.LC_EINVAL
    fake = ctypes.c_void_p(1 << 20)
    # output too small / workspace too small / null count: refused before any launch
    assert lc.lib.lc_setop(lc.SETOP_UNION, fake, P(a), fake, P(b), fake, 1 << 30, fake, a.n + b.n - 1, fake,
                           None) == lc.LC_ENOSPC
    assert lc.lib.lc_setop(lc.SETOP_UNION, fake, P(a), fake, P(b), fake, 16, fake, a.n + b.n, fake,
                           None) == lc.LC_ENOSPC
    assert lc.lib.lc_setop(lc.SETOP_INTERSECT, fake, P(a), fake, P(b), fake, 1 << 30, fake, 1 << 20, None,
                           None) == lc.LC_EINVAL
    # quantile: q = 0 and misaligned k; approximate decode: bad range
    assert lc.lib.lc_quantile(fake, P(a), fake, 0, 5, 0, fake, None) == lc.LC_EINVAL
    assert lc.lib.lc_quantile(fake, P(a), ctypes.c_void_p((1 << 20) + 4), 4, 5, 0, fake, None) == lc.LC_EINVAL
    assert lc.lib.lc_decompress_approx(fake, P(a), 5, 4, fake, None) == lc.LC_EINVAL
    assert lc.lib.lc_decompress_approx(fake, P(a), 0, a.n + 1, fake, None) == lc.LC_EINVAL


def test_batch_and_plan(lc):
    """lc_batch_and_plan is host code: probe = the shorter list (a on ties),
    key and block offsets are prefix sums of the probe lists."""
    lengths = [0, 5, 1024, 1025, 100_000, 3]
    p, t = lc.batch_plan(lengths, 7, 4)

    class B:  # the two fields batch_and_plan reads
        params, table = p, t
    pairs = [(1, 2), (2, 1), (4, 3), (0, 4), (5, 5)]
    table, (tk, tb, ws) = lc.batch_and_plan(B, pairs)
    probe = [1, 1, 3, 0, 5]
    assert list(table["probe"]) == probe
    assert list(table["target"]) == [2, 2, 4, 4, 5]
    n = [lengths[i] for i in probe]
    assert list(table["n"]) == n
    assert list(table["key_off"]) == list(np.concatenate([[0], np.cumsum(n)[:-1]]))
    nb = [-(-x // 1024) for x in n]
    assert list(table["block_off"]) == list(np.concatenate([[0], np.cumsum(nb)[:-1]]))
    assert tk == sum(n) and tb == sum(nb) and ws >= tk * 13
    with pytest.raises(lc.LcError):
        lc.batch_and_plan(B, [(0, 6)])


def _declaration_comments():
    """{name: the comment block right above its declaration} for every
    lc_status entry point of include/lc.h."""
    text = open(os.path.join(ROOT, "include", "lc.h")).read()
    out = {}
    for m in re.finditer(r"/\*((?:(?!\*/).)*)\*/\s*\n\s*lc_status\s+(lc_\w+)\s*\(", text, re.S):
        out[m.group(2)] = m.group(1)
    return out


def test_every_entry_point_cites_the_passage_or_the_callers_it_serves():
    """Each lc_status declaration's comment names the passage of the paper
    that defines its operation (a Def. or a Sec.), or -- for an entry point
    that exists for callers rather than for an operation of the paper --
    the callers it is for."""
    comments = _declaration_comments()
    declared = [n for n in _declared() if n != "lc_strerror"]
    assert sorted(comments) == sorted(declared)
    for name, c in comments.items():
        assert re.search(r"\b(Def\.|Sec\.)\s*[0-9IV]", c) or "callers" in c, name
    # the passages the boundary's core calls follow
    assert "Def. 1" in comments["lc_access"] and "Sec. II-B" in comments["lc_access"]
    assert "Def. 1" in comments["lc_decompress_range"]
    assert "Sec. II-A" in comments["lc_compress_bound"] and "Sec. II-A" in comments["lc_info"]
