"""The request server on the GPU: every result equals the plain definition
(K[a:b], K[i], searchsorted(K, q, 'left')) computed on the host from the same
keys, and is byte-for-byte the same whether the request is served alone (one
request per launch, one launch in flight) or mixed with others (batched
launches overlapping on several streams, arena under pressure)."""
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


@pytest.fixture(scope="module")
def store(lc, wl):
    keys = wl.lognormal_gaps(3_000_000, seed=wl.SEED_BASE + 50, device=DEV)
    blob = lc.compress(keys, 255)
    return keys, wl.as_numpy(keys), blob


def _dest(lc, op, a, b, kb):
    """One device buffer holding every request's result at a 16-byte aligned offset."""
    span = np.where(b > a, b.astype(np.int64) - a.astype(np.int64), 0)
    size = np.where(op == lc.OP_RANGE, span * kb, np.where(op == lc.OP_ACCESS, kb, 8)).astype(np.int64)
    off = np.concatenate([[0], np.cumsum((size + 15) // 16 * 16)[:-1]]).astype(np.int64)
    buf = torch.zeros(int(off[-1] + size[-1] + 16), dtype=torch.uint8, device=DEV)
    return buf, off, size


def _check_results(lc, host, buf, off, size, op, a, b, kb):
    data = buf.cpu().numpy()
    dt = np.uint32 if kb == 4 else np.uint64
    for i in range(len(op)):
        got = data[off[i]:off[i] + size[i]]
        if op[i] == lc.OP_RANGE:
            assert np.array_equal(got.view(dt), host[a[i]:b[i]]), ("range", i, a[i], b[i])
        elif op[i] == lc.OP_ACCESS:
            assert got.view(dt)[0] == host[a[i]], ("access", i, a[i])
        else:
            assert got.view(np.uint64)[0] == np.searchsorted(host, dt(a[i]), side="left"), ("lower_bound", i, a[i])


def _serve(lc, blob, op, a, b, arrival, max_batch, max_inflight, arena_bytes=64 << 20):
    kb = blob.key_bytes
    buf, off, size = _dest(lc, op, a, b, kb)
    req = lc.requests(op, a, b, arrival, buf.data_ptr() + off)
    with lc.Server(blob, arena_bytes, max_batch, max_inflight) as srv:
        res, st = srv.run(req)
    torch.cuda.synchronize()
    return buf, off, size, res, st


@pytest.mark.parametrize("qps", [None, 200_000])
def test_mixed_stream_matches_definitions_and_alone(lc, wl, store, qps):
    keys, host, blob = store
    n = len(host)
    op, a, b, arrival = wl.request_stream(1500, n, int(host[0]), int(host[-1]) + 5, qps, seed=11, max_len=100_000)
    _say(f"serve mixed qps={qps}: {len(op)} requests")
    buf, off, size, res, st = _serve(lc, blob, op, a, b, arrival, max_batch=256, max_inflight=4)
    assert np.all(res["status"] == 0)
    assert np.all(res["complete_ns"] >= res["launch_ns"]) and np.all(res["launch_ns"] >= res["admit_ns"])
    assert np.all(res["admit_ns"] >= arrival.astype(np.int64))
    assert st["launches"] >= 1 and st["max_batch_seen"] <= 256
    _check_results(lc, host, buf, off, size, op, a, b, 8)
    # alone: one request per launch, one launch in flight
    _say("serve alone")
    buf1, _, _, res1, st1 = _serve(lc, blob, op, a, b, np.zeros_like(arrival), max_batch=1, max_inflight=1)
    assert np.all(res1["status"] == 0) and st1["launches"] == len(op) and st1["max_batch_seen"] == 1
    assert torch.equal(buf1, buf)


def test_arena_pressure_keeps_results(lc, wl, store):
    keys, host, blob = store
    n = len(host)
    op, a, b, _ = wl.request_stream(600, n, int(host[0]), int(host[-1]), None, seed=12, max_len=20_000)
    _say("serve with a 256 KB arena")
    buf, off, size, res, st = _serve(lc, blob, op, a, b, np.zeros(len(op), np.uint64), max_batch=64,
                                     max_inflight=3, arena_bytes=256 << 10)
    assert np.all(res["status"] == 0)
    assert st["arena_waits"] > 0 and st["peak_arena_bytes"] <= 256 << 10
    _check_results(lc, host, buf, off, size, op, a, b, 8)


def test_request_errors_and_edges(lc, store):
    keys, host, blob = store
    n = len(host)
    op = np.array([1, 1, 1, 2, 2, 9, 3, 3, 1, 1], dtype=np.uint32)
    a = np.array([5, n - 3, 10, n - 1, n, 0, 0, 2 ** 64 - 1, 7, 0], dtype=np.uint64)
    b = np.array([5, n, 5, 0, 0, 0, 0, 0, n + 1, 40_000], dtype=np.uint64)
    _say("serve errors")
    buf, off, size = _dest(lc, np.where(op > 3, 2, op), a, b, 8)
    req = lc.requests(op, a, b, None, buf.data_ptr() + off)
    with lc.Server(blob, 64 << 10, 8, 2) as srv:  # 64 KB arena: the 40000-key range does not fit
        res, _ = srv.run(req)
    torch.cuda.synchronize()
    want = [0, 0, lc.LC_EINVAL, 0, lc.LC_EINVAL, lc.LC_EINVAL, 0, 0, lc.LC_EINVAL, lc.LC_ENOSPC]
    assert list(res["status"]) == want
    data = buf.cpu().numpy()
    assert np.array_equal(data[off[1]:off[1] + 24].view(np.uint64), host[n - 3:n])
    assert data[off[3]:off[3] + 8].view(np.uint64)[0] == host[n - 1]
    assert data[off[6]:off[6] + 8].view(np.uint64)[0] == 0
    assert data[off[7]:off[7] + 8].view(np.uint64)[0] == n


def test_u32_store_unaligned_ranges(lc, wl):
    keys = wl.uniform_gaps(200_000, seed=13, device=DEV)
    host = wl.as_numpy(keys)
    blob = lc.compress(keys, 63)
    rng = np.random.default_rng(14)
    m = 400
    op = rng.choice([1, 1, 1, 2, 3], m).astype(np.uint32)
    a = rng.integers(0, len(host) - 1, m).astype(np.uint64)
    b = np.minimum(a + rng.integers(1, 5000, m).astype(np.uint64), len(host)).astype(np.uint64)
    lbq = op == 3
    a[lbq] = rng.integers(0, int(host[-1]) + 3, int(lbq.sum()))
    _say("serve u32 store")
    buf, off, size, res, st = _serve(lc, blob, op, a, b, np.zeros(m, np.uint64), max_batch=128, max_inflight=2)
    assert np.all(res["status"] == 0)
    _check_results(lc, host, buf, off, size, op, a, b, 4)


@pytest.mark.parametrize("F", [0, 20])
def test_optimal_fit_store(lc, wl, F):
    """A store compressed with the optimal fit (free intercepts; fraction
    array at F = 20, none at F = 0): mixed requests served in batches equal
    the definitions and the same requests served one by one."""
    keys = wl.lognormal_gaps(400_000, seed=wl.SEED_BASE + 51, device=DEV)
    host = wl.as_numpy(keys)
    blob = lc.compress(keys, 63, frac_bits=F, fit="opt")
    assert blob.info.flags == 1
    rng = np.random.default_rng(15 + F)
    m = 600
    op = rng.choice([1, 1, 2, 3], m).astype(np.uint32)
    a = rng.integers(0, len(host) - 1, m).astype(np.uint64)
    b = np.minimum(a + rng.integers(1, 20_000, m).astype(np.uint64), len(host)).astype(np.uint64)
    lbq = op == 3
    a[lbq] = rng.integers(0, int(host[-1]) + 3, int(lbq.sum())).astype(np.uint64)
    _say(f"serve optimal-fit store F={F}")
    arrival = np.zeros(m, np.uint64)
    buf, off, size, res, st = _serve(lc, blob, op, a, b, arrival, max_batch=256, max_inflight=3)
    assert np.all(res["status"] == 0)
    _check_results(lc, host, buf, off, size, op, a, b, 8)
    alone, _, _, res1, _ = _serve(lc, blob, op, a, b, arrival, max_batch=1, max_inflight=1)
    assert np.all(res1["status"] == 0)
    assert torch.equal(alone, buf)
