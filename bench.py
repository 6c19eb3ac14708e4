"""Benchmark of the learned compressor's hot path on one MI355X.

Workload: 100,000,000 sorted distinct uint64 keys, floor(2^40 x / M) with
x ~ lognormal(0, 2) (M the largest of the first 1e8 draws), de-duplicated;
blocks of 1024 keys; eps swept over {15, 63, 255}.  One step is the whole
path: for every eps, compress (fit + pack + scan + emit) and decompress;
then, on the eps = 63 blob, one decompress_range over the middle half of the
keys, 10M random access(i) and 1M lower_bound(q) with q uniform over the key
range.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  `value` is decoded GB/s = sum(n * 8) / sum(decode
kernel time) over the eps sweep, each decode timed with HIP events on the
stream it runs on.  The CPU baseline times the oracle's plain C decoder on
a bounded prefix of the same keys, single-threaded.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decoded GB/s + lookups/s vs plain per-list kernel; comp. ratio; p99 latency"
HBM_PEAK_GBPS = 8000.0
CALIB_COPY_BYTES = 256 << 20  # plain device copy of known size, read by counter runs to scale them
FLUSH_BYTES = 512 << 20  # each cold decode follows a copy of this many bytes (2x the on-die cache)
HEADLINE_MAX_BYTES = 2048  # the last stdout line (the headline) stays this short
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "decode_traffic.json")
VALU_FILE = os.path.join(ROOT, "profiles", "compress_valu.json")
# VALU peak in lane-operations: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64
# instruction is 64 lane-operations issued over 4 cycles on a 16-lane SIMD)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
KERNEL_SRC = os.path.join(ROOT, "paper_2412_10770_amd", "csrc", "lc_kernels.hip")


def kernel_src_hash() -> str:
    import hashlib
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def recorded_traffic():
    """HBM bytes per decompress call from the committed counter runs, or None
    when the kernels changed since they were taken."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_src_sha256_16") != kernel_src_hash():
        return None
    return rec


def recorded_valu():
    """VALU instructions per lc_compress call (all its kernels) from the
    committed counter run, or None when the kernels changed since."""
    try:
        rec = json.load(open(VALU_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_src_sha256_16") != kernel_src_hash():
        return None
    return rec


# Fractional bits F of the fixed-point slopes in every measured blob
# (--frac-bits).  0, integer slopes, gives smaller blobs and equal or faster
# decode than 20 on every workload measured here; bench_fits reports both.
FRAC_BITS = 0


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cpu():
    """The host's CPU model (from /proc/cpuinfo) and the cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def cpu_baseline(host_keys, eps_list, budget_s: float = 24.0, max_threads: int = 16, reps: int = 5):
    """The oracle's plain C decoder timed on the host over the same eps sweep
    as the step, on a sample of the workload (whole blocks spread over the
    list) sized to about budget_s seconds of oracle work.  Single core: the
    sample as one blob per eps.  All cores: the sample split at block
    boundaries into one piece per thread (runs dealt round-robin),
    each piece compressed by the oracle into its own blob and the blobs
    decoded concurrently (the oracle is called through ctypes, which releases
    the interpreter lock, so the threads run in parallel).  Each figure is the
    median of `reps` runs after one warm-up; value = sum(8 n) / sum over eps
    of the all-core median.  Point queries at the middle eps of the sweep:
    the oracle answers a batch of access(i) (i uniform) or lower_bound(q)
    (q uniform over the keys' range) by decoding the blob and applying the
    plain definition; all cores: each thread answers its own piece's share of
    the batch from that piece's blob."""
    import statistics
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import oracle
    from paper_2412_10770_amd import workloads

    model, avail = host_cpu()
    threads = max(1, min(max_threads, avail))

    def spread(m: int, chunks: int = 64):
        """About m keys as `chunks` block-aligned runs of whole 1024-key blocks spread evenly over
        the keys (so the sample has the whole range's mix of dense and sparse blocks, and its
        blocks are blocks of the full list); all keys (cut into runs) when m reaches their number."""
        n = len(host_keys)
        run = max(1024, (m // chunks) & ~1023)
        if run * chunks >= n:
            cuts = [(n * c // chunks) & ~1023 for c in range(chunks)] + [n]
            return [host_keys[a:b] for a, b in zip(cuts, cuts[1:]) if b > a]
        starts = [(int(s) & ~1023) for s in np.linspace(0, n - run, chunks)]
        return [host_keys[s:s + run] for s in starts]

    probe = np.ascontiguousarray(np.concatenate(spread(64 * 1024)))
    blob = oracle.compress(probe, eps_list[0], 10, FRAC_BITS)
    t0 = time.perf_counter()
    oracle.decode(blob)
    per_key = (time.perf_counter() - t0) / len(probe)
    # per eps: one compress (about a decode's time) + (1 + reps) single-core decodes, then the
    # same on all cores (a fraction of that)
    # + two query batches, each (1 + reps) decodes of the sample on one core and on all cores
    units = (len(eps_list) * (2 + reps) + 2 * (1 + reps)) * (1.0 + 2.0 / threads)
    runs = spread(int(budget_s / units / max(per_key, 1e-9)))
    sample = np.ascontiguousarray(np.concatenate(runs))
    n_s = len(sample)
    # thread t takes runs t, t + threads, ... (in order, so each piece is a sorted list of whole
    # blocks): every piece gets a share of the dense and of the sparse stretches
    pieces = [np.ascontiguousarray(np.concatenate(runs[t::threads])) for t in range(min(threads, len(runs)))]

    def median_time(fn):
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts)

    q_eps = eps_list[len(eps_list) // 2]
    one_dec = one_enc = all_dec = all_enc = 0.0
    with ThreadPoolExecutor(max_workers=len(pieces)) as pool:
        for eps in eps_list:
            t0 = time.perf_counter()
            blob = oracle.compress(sample, eps, 10, FRAC_BITS)
            one_enc += time.perf_counter() - t0
            assert np.array_equal(oracle.decode(blob), sample)
            one_dec += median_time(lambda: oracle.decode(blob))
            t0 = time.perf_counter()
            pblobs = list(pool.map(lambda k: oracle.compress(k, eps, 10, FRAC_BITS), pieces))
            all_enc += time.perf_counter() - t0
            all_dec += median_time(lambda: list(pool.map(oracle.decode, pblobs)))
            if eps == q_eps:
                q_blob, q_pblobs = blob, pblobs

        # point queries: one batch of n_q over the sample; on all cores piece t takes n_q / pieces of
        # them, drawn over its own indices and key range
        n_q = 1 << 20
        share = n_q // len(pieces)
        idx = workloads.uniform_indices(n_q, n_s, seed=workloads.SEED_BASE + 202).numpy()
        qk = workloads.uniform_keys(n_q, int(sample[0]), int(sample[-1]), seed=workloads.SEED_BASE + 203).numpy()
        p_idx = [workloads.uniform_indices(share, len(k), seed=workloads.SEED_BASE + 204 + t).numpy()
                 for t, k in enumerate(pieces)]
        p_q = [workloads.uniform_keys(share, int(k[0]), int(k[-1]), seed=workloads.SEED_BASE + 204 + t).numpy()
               for t, k in enumerate(pieces)]
        assert np.array_equal(oracle.access(oracle.decode(q_blob), idx), sample[idx])
        assert np.array_equal(oracle.lower_bound(oracle.decode(q_blob), qk).astype(np.int64),
                              np.searchsorted(sample, qk.astype(sample.dtype)))
        one_acc = median_time(lambda: oracle.access(oracle.decode(q_blob), idx))
        one_lb = median_time(lambda: oracle.lower_bound(oracle.decode(q_blob), qk))
        pt = range(len(pieces))
        all_acc = median_time(lambda: list(pool.map(lambda t: oracle.access(oracle.decode(q_pblobs[t]), p_idx[t]), pt)))
        all_lb = median_time(lambda: list(pool.map(lambda t: oracle.lower_bound(oracle.decode(q_pblobs[t]), p_q[t]),
                                                   pt)))
    nb = n_s * 8 * len(eps_list)
    n_all = share * len(pieces)
    eps_s = "/".join(str(e) for e in eps_list)
    return {
        "value": round(nb / all_dec / 1e9, 4), "unit": "GB/s", "cores": len(pieces), "kind": "oracle",
        "sample": f"{n_s} keys (64 block-aligned runs spread over the list), eps {eps_s}: oracle decode, "
                  f"{len(pieces)} threads on block-aligned pieces, median of {reps} after 1 warm-up",
        "single_core_GBps": round(nb / one_dec / 1e9, 4),
        "compress_GBps": {"single_core": round(nb / one_enc / 1e9, 4), "all_cores": round(nb / all_enc / 1e9, 4)},
        "access_lookups_per_s": {"single_core": round(n_q / one_acc, 1), "all_cores": round(n_all / all_acc, 1)},
        "lower_bound_lookups_per_s": {"single_core": round(n_q / one_lb, 1), "all_cores": round(n_all / all_lb, 1)},
        "queries": f"eps {q_eps}: {n_q} access(i), i uniform, and {n_q} lower_bound(q), q uniform over the "
                   f"sample's key range, each batch answered by an oracle decode of the blob and the plain "
                   f"definition; all cores: {share} of each per piece from its own blob",
        "host": {"cpu": model, "cores_available": avail, "nproc": os.cpu_count()},
    }


def bench_batch(dev, steps: int, warmup: int, nlists: int = 4096, cands=(7, 31, 127)):
    """Posting-list batch: nlists uint32 lists (lengths from the power law
    L^-1.1 on [100, 10^6], geometric gaps of per-list mean log-uniform in
    [2, 2000]).  Batched: one size pass over the eps candidates, the on-device
    pick, compress and decompress, each one launch (or a few) over all lists.
    Per list: lc_compress + lc_decompress launched once per list at the eps
    the autotuner chose, so both sides produce identical blobs.  Each side is
    timed eagerly and replayed from a captured hipGraph."""
    import numpy as np
    import torch

    from paper_2412_10770_amd import lc, workloads

    t0 = time.perf_counter()
    keys, lengths = workloads.posting_lists(nlists, device=dev)
    torch.cuda.synchronize()
    n = keys.numel()
    log(f"batch: generated {nlists} lists, {n} keys in {time.perf_counter() - t0:.1f} s")
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    p, table = lc.batch_plan(lengths, cands[0], 4, max(cands), frac_bits=FRAC_BITS)
    d_lists = torch.from_numpy(table.view(np.uint8).copy()).to(dev)
    ws = torch.empty(p.ws_bytes, dtype=torch.uint8, device=dev)
    blob = torch.empty(p.blob_bytes, dtype=torch.uint8, device=dev)
    sizes = torch.empty(nlists, dtype=torch.int64, device=dev)
    csizes = torch.empty(len(cands) * nlists, dtype=torch.int64, device=dev)
    stats = torch.zeros(2, dtype=torch.int32, device=dev)
    dstats = torch.zeros(1, dtype=torch.int32, device=dev)
    out = torch.empty(n, dtype=torch.int32, device=dev)

    # first pass, eager: learns the eps picked per list and the largest segment area
    lc.batch_sizes_async(keys, d_lists, p, cands, ws, csizes, stats)
    lc.batch_pick_eps_async(d_lists, p, csizes, cands)
    lc.batch_compress_async(keys, d_lists, p, blob, ws, sizes, stats)
    st = stats.cpu().numpy()
    assert st[0] == 0, f"batch compress flags {st[0]}"
    max_seg = int(st[1])
    lc.batch_decompress_async(blob, d_lists, p, max_seg, out, dstats)
    assert torch.equal(out, keys) and int(dstats.item()) == 0, "batch round trip failed"
    chosen = d_lists.cpu().numpy().view(lc.BATCH_LIST_DTYPE)["eps"].copy()
    bsizes = sizes.cpu().numpy()
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def mark(marks, i):
        if marks is not None:
            marks[i].record()

    def batched(marks):
        stats.zero_()
        dstats.zero_()
        mark(marks, 0)
        lc.batch_sizes_async(keys, d_lists, p, cands, ws, csizes, stats)
        lc.batch_pick_eps_async(d_lists, p, csizes, cands)
        mark(marks, 1)
        lc.batch_compress_async(keys, d_lists, p, blob, ws, sizes, stats)
        mark(marks, 2)
        lc.batch_decompress_async(blob, d_lists, p, max_seg, out, dstats)
        mark(marks, 3)

    # per-list launches into the same slot layout of a second buffer
    blob2 = torch.empty(p.blob_bytes, dtype=torch.uint8, device=dev)
    ws2 = torch.empty(max(16, max(lc.compress_bound(int(m), 4, int(e), frac_bits=FRAC_BITS)[1] for m, e in zip(lengths, chosen))),
                      dtype=torch.uint8, device=dev)
    nb2 = torch.zeros(nlists, dtype=torch.int64, device=dev)
    fl2 = torch.zeros(1, dtype=torch.int32, device=dev)
    out2 = torch.empty(n, dtype=torch.int32, device=dev)
    kviews = [keys[o:o + m] for o, m in zip(offs, lengths)]
    oviews = [out2[o:o + m] for o, m in zip(offs, lengths)]
    bviews = [blob2[int(table["blob_off"][l]):int(table["blob_off"][l] + table["blob_cap"][l])] for l in range(nlists)]
    for l in range(nlists):
        lc.compress_async(kviews[l], int(chosen[l]), bviews[l], ws2, nb2[l:l + 1], fl2, frac_bits=FRAC_BITS)
    torch.cuda.synchronize()
    assert int(fl2.item()) == 0
    infos = [lc.Blob.from_device(bviews[l]) for l in range(nlists)]
    assert np.array_equal(nb2.cpu().numpy(), bsizes), "per-list blob sizes differ from the batch's"

    def per_list(marks):
        mark(marks, 0)
        for l in range(nlists):
            lc.compress_async(kviews[l], int(chosen[l]), bviews[l], ws2, nb2[l:l + 1], fl2, frac_bits=FRAC_BITS)
        mark(marks, 1)
        for l in range(nlists):
            lc.decompress(infos[l], out=oviews[l])
        mark(marks, 2)

    def run(fn, nmarks, reps, graph, o):
        g = None
        if graph:
            fn(None)  # warm (kernel attributes set outside the capture)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                fn(None)
        else:
            for _ in range(warmup):
                fn(None)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            o.zero_()  # every run / replay must rewrite the whole output
            a, b = ev(), ev()
            marks = None if graph else [ev() for _ in range(nmarks)]
            a.record()
            if graph:
                g.replay()
            else:
                fn(marks)
            b.record()
            torch.cuda.synchronize()
            assert torch.equal(o, keys), f"round trip failed ({'graph replay' if graph else 'eager'})"
            times.append((a.elapsed_time(b), [m0.elapsed_time(m1) for m0, m1 in zip(marks, marks[1:])]
                          if marks else None))
        return g, times

    res = {}
    for name, fn, nm, reps in (("batched", batched, 4, steps), ("per_list", per_list, 3, max(2, steps // 4))):
        for graph in (False, True):
            log(f"batch: timing {name} {'graph' if graph else 'eager'}")
            g, times = run(fn, nm, reps, graph, out if name == "batched" else out2)
            total = float(np.mean([t[0] for t in times]))
            entry = {"ms": round(total, 3)}
            if not graph:
                ph = np.mean([t[1] for t in times], axis=0)
                if name == "batched":
                    entry.update(autotune_ms=round(float(ph[0]), 3), compress_ms=round(float(ph[1]), 3),
                                 decompress_ms=round(float(ph[2]), 3))
                else:
                    entry.update(compress_ms=round(float(ph[0]), 3), decompress_ms=round(float(ph[1]), 3))
            res[f"{name}_{'graph' if graph else 'eager'}"] = entry
            del g
    b, pl = res["batched_eager"], res["per_list_eager"]
    key_bytes = n * 4
    # block size picked by the autotuner: exact bytes and decode time per size
    log("batch: block-size and fit autotune")
    fits = (("greedy", 0), ("greedy", 20), ("opt", 0), ("opt", 20))
    _, tune = lc.autotune_batch(keys, lengths, cands, block_candidates=(8, 9, 10, 11, 12), objective="size",
                                frac_bits=FRAC_BITS, fit_candidates=fits)
    row = lambda r: {"log2_block": r["log2_block"], "fit": r["fit"], "frac_bits": r["frac_bits"],  # noqa: E731
                     "bits_per_key": round(8.0 * r["bytes"] / n, 4),
                     "decode_GBps": round(key_bytes / r["decode_ms"] / 1e6, 2), "chosen": r["chosen"]}
    block_tune = [row(r) for r in tune if r["fit"] == "greedy" and r["frac_bits"] == FRAC_BITS]
    picked = next(r for r in tune if r["chosen"])
    lb_best = picked["log2_block"]
    ref = next(r for r in tune if r["log2_block"] == lb_best and r["fit"] == "greedy" and r["frac_bits"] == FRAC_BITS)
    fit_tune = [dict(row(r), bytes_saved_pct_vs_greedy=round(100.0 * (ref["bytes"] - r["bytes"]) / ref["bytes"], 3))
                for r in tune if r["log2_block"] == lb_best]
    tiling_tune = {"log2_block": picked["log2_block"], "tiling": picked.get("tiling"),
                   "compress_ms": {k: round(v, 3) for k, v in picked.get("compress_ms_by_tiling", {}).items()}}
    return {
        "workload": f"{nlists} sorted uint32 lists, lengths ~ L^-1.1 on [100, 1e6] ({n} keys), geometric gaps "
                    f"with per-list mean log-uniform in [2, 2000]; eps per list argmin-size over {list(cands)}; "
                    f"F = {FRAC_BITS}",
        "n": n, "nlists": nlists,
        "ratio": round(float(bsizes.sum()) / key_bytes, 5),
        "bits_per_key": round(8.0 * float(bsizes.sum()) / n, 4),
        "eps_chosen": {str(c): int((chosen == c).sum()) for c in cands},
        "lists_expanding": int((bsizes > lengths * 4).sum()),
        "decoded_GBps": {"batched": round(key_bytes / b["decompress_ms"] / 1e6, 2),
                         "per_list": round(key_bytes / pl["decompress_ms"] / 1e6, 2)},
        "compress_GBps": {"batched": round(key_bytes / b["compress_ms"] / 1e6, 2),
                          "per_list": round(key_bytes / pl["compress_ms"] / 1e6, 2)},
        "step_ms": {k: v["ms"] for k, v in res.items()},
        "phases_ms": {k: {kk: vv for kk, vv in v.items() if kk != "ms"} for k, v in res.items() if "eager" in k},
        "block_size_autotune": block_tune,
        "fit_autotune": fit_tune,
        "tiling_autotune": tiling_tune,
        "note": "batched step = autotune (size pass over the candidates + pick) + compress + decompress; "
                "per-list step = compress + decompress only (eps given), identical blobs; the step runs at "
                "1024-key blocks, block_size_autotune reports the tuner's sweep (objective: fewest bytes)",
    }


def bench_small(dev, n: int = 1_000_000, eps: int = 63, n_access: int = 100_000, reps: int = 20):
    """The plain-method configuration: n sorted uint32 keys, gaps uniform in
    [1, 64], eps 63, 1024-key blocks: compress + decompress + n_access
    access(i) with i uniform, each timed with HIP events (mean of reps after
    one warm-up), beside the CPU oracle on the same keys (compress, decode).
    Small enough that launches and the per-block walk, not bandwidth, set
    the time."""
    import numpy as np
    import torch

    import oracle
    from paper_2412_10770_amd import lc, workloads

    keys = workloads.uniform_gaps(n, device=dev)
    host = workloads.as_numpy(keys)
    idx = workloads.uniform_indices(n_access, n, seed=workloads.SEED_BASE + 106, device=dev)
    bmax, wsb = lc.compress_bound(n, 4, eps, frac_bits=FRAC_BITS)
    blob = torch.empty(bmax, dtype=torch.uint8, device=dev)
    ws = torch.empty(max(wsb, 16), dtype=torch.uint8, device=dev)
    nb = torch.zeros(1, dtype=torch.int64, device=dev)
    fl = torch.zeros(1, dtype=torch.int32, device=dev)
    lc.compress_async(keys, eps, blob, ws, nb, fl, frac_bits=FRAC_BITS)
    torch.cuda.synchronize()
    b = lc.Blob.from_device(blob)
    out = lc.decompress(b)
    acc = lc.access(b, idx)
    assert torch.equal(out, keys) and torch.equal(acc, keys[idx])
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    tc, td, ta = [], [], []
    for _ in range(reps + 1):
        e0, e1, e2, e3 = ev(), ev(), ev(), ev()
        e0.record()
        lc.compress_async(keys, eps, blob, ws, nb, fl, frac_bits=FRAC_BITS)
        e1.record()
        lc.decompress(b, out=out)
        e2.record()
        lc.access(b, idx, out=acc, flags=fl, check=False)
        e3.record()
        torch.cuda.synchronize()
        tc.append(e0.elapsed_time(e1))
        td.append(e1.elapsed_time(e2))
        ta.append(e2.elapsed_time(e3))
    assert int(fl.item()) == 0
    import time
    t0 = time.perf_counter()
    ob = oracle.compress(host, eps, 10, FRAC_BITS)
    t_oc = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.decode(ob)
    t_od = time.perf_counter() - t0
    assert np.array_equal(ob, b.data.cpu().numpy())
    c, d_, a_ = float(np.mean(tc[1:])), float(np.mean(td[1:])), float(np.mean(ta[1:]))
    return {
        "workload": f"{n} sorted uint32 keys, K[0] = 0, gaps uniform in [1, 64]; eps {eps}, blocks of 1024, "
                    f"F = {FRAC_BITS}; compress + decompress + {n_access} access(i), i uniform",
        "bits_per_key": round(b.bits_per_key, 4), "ratio": round(b.ratio, 5),
        "compress_ms": round(c, 4), "decompress_ms": round(d_, 4),
        "decoded_GBps": round(n * 4 / d_ / 1e6, 2), "access_lookups_per_s": round(n_access / a_ * 1e3, 1),
        "step_ms": round(c + d_ + a_, 4),
        "oracle_cpu_one_core": {"compress_ms": round(t_oc * 1e3, 2), "decode_ms": round(t_od * 1e3, 2)},
        "note": "the GPU blob equals the oracle's byte for byte",
    }


def bench_lookups(dev, n: int = 200_000_000, eps: int = 63, n_access: int = 10_000_000, n_lb: int = 1_000_000,
                  reps: int = 10):
    """Point lookups on the heterogeneous-runs workload: n uint64 keys in
    alternating dense (gaps 1..4) and Zipf(1.2) runs; eps 63; n_access
    access(i) with i uniform and n_lb lower_bound(q) with q uniform over the
    key range, each batch one launch timed with HIP events."""
    import numpy as np
    import torch

    from paper_2412_10770_amd import lc, workloads

    keys = workloads.heterogeneous_runs(n, device=dev)
    blob = lc.compress(keys, eps, frac_bits=FRAC_BITS)
    idx = workloads.uniform_indices(n_access, n, seed=workloads.SEED_BASE + 104, device=dev)
    q = workloads.uniform_keys(n_lb, int(keys[0]), int(keys[-1]), seed=workloads.SEED_BASE + 105, device=dev)
    acc = lc.access(blob, idx)
    pos = lc.lower_bound(blob, q)
    assert torch.equal(acc, keys[idx]) and torch.equal(pos, torch.searchsorted(keys, q, side="left"))
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    ta, tl = [], []
    for _ in range(reps):
        e0, e1, e2 = ev(), ev(), ev()
        e0.record()
        lc.access(blob, idx, out=acc, flags=flags, check=False)
        e1.record()
        lc.lower_bound(blob, q, out=pos)
        e2.record()
        torch.cuda.synchronize()
        ta.append(e0.elapsed_time(e1))
        tl.append(e1.elapsed_time(e2))
    assert int(flags.item()) == 0
    # the same lookups on the uncompressed keys (torch gather / searchsorted), for context
    ua, ul = [], []
    for _ in range(reps):
        e0, e1, e2 = ev(), ev(), ev()
        e0.record()
        torch.index_select(keys, 0, idx, out=acc)
        e1.record()
        torch.searchsorted(keys, q, side="left", out=pos)
        e2.record()
        torch.cuda.synchronize()
        ua.append(e0.elapsed_time(e1))
        ul.append(e1.elapsed_time(e2))
    return {
        "uncompressed_torch": {
            "access_lookups_per_s": round(n_access / float(np.mean(ua)) * 1e3, 1),
            "lower_bound_lookups_per_s": round(n_lb / float(np.mean(ul)) * 1e3, 1),
            "bytes": n * 8,
        },
        "workload": f"{n} uint64 keys, alternating dense (gaps U[1,4]) and Zipf(1.2) runs of 1e4..1e6 keys; "
                    f"eps {eps}, F = {FRAC_BITS}; {n_access} access(i), i uniform; {n_lb} lower_bound(q), q uniform "
                    f"over the key range",
        "bits_per_key": round(blob.bits_per_key, 4),
        "access_lookups_per_s": round(n_access / float(np.mean(ta)) * 1e3, 1),
        "lower_bound_lookups_per_s": round(n_lb / float(np.mean(tl)) * 1e3, 1),
        "access_ms": round(float(np.mean(ta)), 4), "lower_bound_ms": round(float(np.mean(tl)), 4),
    }


def bench_queries(dev, n: int = 100_000_000, eps: int = 63, n_quantile: int = 10_000_000, npairs: int = 48,
                  reps: int = 5):
    """Queries on the compressed form.  On the lognormal store (n keys, eps):
    the approximate decode (model only, no residual slab) against the exact
    decode, and n_quantile quantiles, exact and approximate.  On posting
    lists (the batch workload's recipe): list AND of a short list (1e3..1e4
    keys) with a long one (the longest lists) and list OR of the same pairs,
    each one lc_setop call, against decoding both lists and intersecting /
    merging the decoded keys with torch (searchsorted, masked_select,
    cat + unique)."""
    import numpy as np
    import torch

    from paper_2412_10770_amd import lc, workloads

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = ev(), ev()
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.mean(ts))

    keys = workloads.lognormal_distinct(n, device=dev)
    blob = lc.compress(keys, eps, frac_bits=FRAC_BITS)
    out = torch.empty(n, dtype=torch.int64, device=dev)
    lc.decompress(blob, out=out)
    assert torch.equal(out, keys)
    t_exact = timed(lambda: lc.decompress(blob, out=out))
    t_apx = timed(lambda: lc.decompress_approx(blob, out=out))
    err = int((out - keys).abs().max())
    assert err <= eps
    kq = workloads.uniform_indices(n_quantile, 1 << 20, seed=workloads.SEED_BASE + 106, device=dev)
    qout = torch.empty(n_quantile, dtype=torch.int64, device=dev)
    t_q = timed(lambda: lc.quantile(blob, kq, 1 << 20, out=qout))
    t_qa = timed(lambda: lc.quantile(blob, kq, 1 << 20, approx=True, out=qout))
    del keys, out, blob
    torch.cuda.empty_cache()

    pl, lengths = workloads.posting_lists(4096, device=dev)
    offs = np.concatenate([[0], np.cumsum(lengths)[:-1]])
    rng = np.random.default_rng(workloads.SEED_BASE + 107)
    longs = np.argsort(lengths)[-npairs:]
    shorts = rng.choice(np.flatnonzero((lengths >= 1000) & (lengths <= 10000)), npairs, replace=False)
    pairs = []
    for s_, l_ in zip(shorts, longs):
        a = pl[offs[s_]:offs[s_] + lengths[s_]]
        b = pl[offs[l_]:offs[l_] + lengths[l_]]
        pairs.append((a, b, lc.compress(a, 31, frac_bits=FRAC_BITS), lc.compress(b, 31, frac_bits=FRAC_BITS)))
    del pl
    # buffers sized for the largest pair, allocated once
    mx_and = max(lc.setop_bound(A, B, lc.SETOP_INTERSECT)[1] for _, _, A, B in pairs)
    mx_or = max(lc.setop_bound(A, B, lc.SETOP_UNION) for _, _, A, B in pairs)
    ws = torch.empty(max(mx_and, mx_or[1]), dtype=torch.uint8, device=dev)
    sout = torch.empty(mx_or[0], dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    da = torch.empty(max(int(x[0].numel()) for x in pairs), dtype=torch.int32, device=dev)
    db = torch.empty(max(int(x[1].numel()) for x in pairs), dtype=torch.int32, device=dev)
    u = lambda t: t.to(torch.int64) & 0xFFFFFFFF  # noqa: E731  (uint32 keys held as int32 bit patterns)
    for a, b, A, B in pairs[:4]:  # the timed paths give the definitions' answers
        assert torch.equal(u(lc.intersect(A, B)), u(a)[torch.isin(u(a), u(b))].unique())
        assert torch.equal(u(lc.union(A, B)), torch.cat([u(a), u(b)]).unique())

    def run_and():
        for _, _, A, B in pairs:
            lc.setop_async(lc.SETOP_INTERSECT, A, B, ws, sout, cnt)

    def run_or():
        for _, _, A, B in pairs:
            lc.setop_async(lc.SETOP_UNION, A, B, ws, sout, cnt)

    def base_and():
        for _, _, A, B in pairs:
            x, y = da[:A.n], db[:B.n]
            lc.decompress(A, out=x)
            lc.decompress(B, out=y)
            x, y = u(x), u(y)
            p = torch.searchsorted(y, x).clamp_(max=y.numel() - 1)
            x.masked_select(y[p] == x)

    def base_or():
        for _, _, A, B in pairs:
            x, y = da[:A.n], db[:B.n]
            lc.decompress(A, out=x)
            lc.decompress(B, out=y)
            torch.cat([u(x), u(y)]).unique()

    t_and, t_or = timed(run_and), timed(run_or)
    t_band, t_bor = timed(base_and), timed(base_or)

    # many pairs at once: AND of random pairs of lists of the whole batch
    pl2, _ = workloads.posting_lists(4096, device=dev)
    batch = lc.batch_compress(pl2, lengths, candidates=(7, 31, 127), frac_bits=FRAC_BITS)
    del pl2
    npq = 4096
    qpairs = rng.integers(0, len(lengths), (npq, 2))
    table, totals = lc.batch_and_plan(batch, qpairs)
    d_pairs = torch.from_numpy(table.view(np.uint8).copy()).to(dev)
    bws = torch.empty(max(totals[2], 16), dtype=torch.uint8, device=dev)
    bout = torch.empty(max(totals[0], 1), dtype=torch.int32, device=dev)
    bcnt = torch.zeros(npq, dtype=torch.int64, device=dev)
    bst = torch.zeros(1, dtype=torch.int32, device=dev)
    t_batched = timed(lambda: lc.batch_and_async(batch, d_pairs, npq, totals, bws, bout, bcnt, bst))
    assert int(bst.item()) == 0
    blobs = [batch.blob(l) for l in range(len(lengths))]
    for i in range(8):  # same answers one pair at a time
        a, b = qpairs[i]
        o = int(table["key_off"][i])
        assert torch.equal(lc.intersect(blobs[a], blobs[b]), bout[o:o + int(bcnt[i])])
    pws = torch.empty(max(lc.setop_bound(blobs[a], blobs[b], lc.SETOP_INTERSECT)[1] for a, b in qpairs),
                      dtype=torch.uint8, device=dev)
    pout = torch.empty(int(max(min(lengths[a], lengths[b]) for a, b in qpairs)) + 1, dtype=torch.int32, device=dev)

    def per_pair():
        for a, b in qpairs:
            lc.setop_async(lc.SETOP_INTERSECT, blobs[a], blobs[b], pws, pout, cnt)

    t_per_pair = timed(per_pair)
    short_keys = int(sum(A.n for _, _, A, _ in pairs))
    long_keys = int(sum(B.n for _, _, _, B in pairs))
    return {
        "workload": f"approximate decode and quantiles on {n} lognormal uint64 keys (eps {eps}, F = {FRAC_BITS}); list AND / OR "
                    f"of {npairs} pairs of posting lists (a list of 1e3..1e4 keys with one of the {npairs} longest, "
                    f"eps 31), one call per pair",
        "decode_exact_GBps": round(n * 8 / t_exact / 1e6, 2),
        "decode_approx_GBps": round(n * 8 / t_apx / 1e6, 2),
        "approx_max_error": err,
        "quantiles_per_s": round(n_quantile / t_q * 1e3, 1),
        "approx_quantiles_per_s": round(n_quantile / t_qa * 1e3, 1),
        "and_pairs_per_s": round(npairs / t_and * 1e3, 1),
        "and_pairs_per_s_decode_both_torch": round(npairs / t_band * 1e3, 1),
        "or_pairs_per_s": round(npairs / t_or * 1e3, 1),
        "or_pairs_per_s_decode_both_torch": round(npairs / t_bor * 1e3, 1),
        "and_probe_keys": short_keys, "and_searched_keys": long_keys,
        "batched_and": {"pairs": npq, "probe_keys": int(totals[0]), "ms": round(t_batched, 3),
                        "pairs_per_s": round(npq / t_batched * 1e3, 1),
                        "pairs_per_s_one_call_each": round(npq / t_per_pair * 1e3, 1)},
    }


def bench_serve(dev, n: int = 1_000_000_000, qps_points=(1e3, 1e4, 1e5, 1e6, None), arena_bytes: int = 2 << 30,
                max_batch: int = 1024, max_inflight: int = 4, eps_cands=(15, 63, 255, 1023)):
    """Request server over a compressed store of n uint64 keys (gaps
    max(1, ceil(lognormal(3, 1.5)))), eps = the candidate giving the smallest
    blob.  Poisson request streams at each rate (None: all at time 0, the
    saturation point): 70% decode_range of length floor(exp(U[0, ln 1e6])),
    20% access(i), 10% lower_bound(q).  Latency = completion - scheduled
    arrival.  Unbatched reference: the same server at one request per launch
    and one launch in flight (plain per-request launches, no host overhead)."""
    import numpy as np
    import torch

    from paper_2412_10770_amd import lc, workloads

    t0 = time.perf_counter()
    keys = workloads.lognormal_gaps(n, seed=workloads.SEED_BASE + 5, device=dev)
    torch.cuda.synchronize()
    lo, hi = int(keys[0]), int(keys[-1])
    log(f"serve: generated {n} keys in {time.perf_counter() - t0:.1f} s")
    best = None
    sizes = {}
    for e in eps_cands:
        b = lc.compress(keys, e, frac_bits=FRAC_BITS)
        sizes[e] = b.nbytes
        if best is None or b.nbytes < best.nbytes:
            best = b
        del b
        torch.cuda.empty_cache()
    blob = best
    # the store round-trips (checked in slices to bound the extra memory)
    step = 100_000_000
    for s0 in range(0, n, step):
        e0 = min(n, s0 + step)
        assert torch.equal(lc.decompress_range(blob, s0, e0), keys[s0:e0]), "store round trip failed"
    del keys
    torch.cuda.empty_cache()
    log(f"serve: store eps={blob.info.eps}, {blob.nbytes / 1e9:.3f} GB ({blob.bits_per_key:.3f} bits/key)")

    def point(srv, qps, count, seed):
        op, a, b, arr = workloads.request_stream(count, n, lo, hi, qps, seed=seed)
        res, st = srv.run(lc.requests(op, a, b, arr))
        assert np.all(res["status"] == 0), "request failed"
        lat = (res["complete_ns"] - arr.astype(np.int64)) / 1e3
        span_s = (res["complete_ns"].max() - int(arr.min())) / 1e9
        out_bytes = float(np.where(op == 1, (b - a) * 8, 8).sum())
        return {
            "qps_offered": qps if qps is not None else "saturation",
            "requests": count,
            "p50_us": round(float(np.percentile(lat, 50)), 1),
            "p99_us": round(float(np.percentile(lat, 99)), 1),
            "qps_achieved": round(count / span_s, 1),
            "decoded_GBps": round(float(np.where(op == 1, (b - a) * 8, 0).sum()) / span_s / 1e9, 2),
            "output_GBps": round(out_bytes / span_s / 1e9, 2),
            "launches": st["launches"], "max_batch_seen": st["max_batch_seen"],
            "arena_waits": st["arena_waits"], "peak_arena_MB": round(st["peak_arena_bytes"] / 2 ** 20, 1),
        }

    points = []
    with lc.Server(blob, arena_bytes, max_batch, max_inflight) as srv:
        point(srv, None, 2000, seed=1)  # warm
        for k, qps in enumerate(qps_points):
            count = 100_000 if qps is None else int(min(100_000, max(1000, qps * 0.25)))
            log(f"serve: qps={qps or 'saturation'} ({count} requests)")
            points.append(point(srv, qps, count, seed=100 + k))
    with lc.Server(blob, arena_bytes, 1, 1) as srv:
        log("serve: unbatched reference at saturation")
        unb = point(srv, None, 20_000, seed=200)
    sat = points[-1]
    return {
        "workload": f"{n} sorted uint64 keys, gaps max(1, ceil(lognormal(3, 1.5))); store eps argmin-size over "
                    f"{list(eps_cands)}, F = {FRAC_BITS}; Poisson arrivals, 70% decode_range (length floor(exp(U[0, ln 1e6]))), "
                    f"20% access, 10% lower_bound; output arena {arena_bytes >> 20} MiB, "
                    f"{max_batch} requests per launch, {max_inflight} launches in flight",
        "store": {"eps": blob.info.eps, "bytes": blob.nbytes, "bits_per_key": round(blob.bits_per_key, 4),
                  "bytes_by_eps": {str(e): v for e, v in sizes.items()}},
        "points": points,
        "unbatched_saturation": unb,
        "saturation_speedup_vs_unbatched": round(sat["qps_achieved"] / unb["qps_achieved"], 2),
    }


def bench_fits(dev, keys_lognormal=None, reps: int = 3):
    """The fits side by side: greedy, fewest anchored segments ("min") and
    the optimal free-intercept fit ("opt") at F = 20, and greedy and opt at
    F = 0 (integer slopes and intercepts: no fraction array).  Compress and
    decompress time (HIP events, mean of `reps` after one warm-up), blob size
    and segment count, per workload and eps.  Every blob is decoded and
    compared with its keys; 1e6 access(i) and 1e6 lower_bound(q) (uniform)
    are timed on it and compared with the definitions."""
    import numpy as np
    import torch

    from paper_2412_10770_amd import lc, workloads

    def ev():
        return torch.cuda.Event(enable_timing=True)

    cases = [
        ("lognormal_distinct_100M_u64", lambda: keys_lognormal if keys_lognormal is not None
         else workloads.lognormal_distinct(100_000_000, device=dev), (15, 63, 255)),
        ("uniform_gaps_100M_u32", lambda: workloads.uniform_gaps(100_000_000, device=dev), (7, 31, 127)),
        ("lognormal_gaps_100M_u64", lambda: workloads.lognormal_gaps(100_000_000, device=dev), (63, 255, 1023)),
        ("heterogeneous_runs_200M_u64", lambda: workloads.heterogeneous_runs(200_000_000, device=dev), (63,)),
    ]
    variants = (("greedy", "greedy", 20), ("min", "min", 20), ("opt", "opt", 20),
                ("greedy_F0", "greedy", 0), ("opt_F0", "opt", 0))
    res = {}
    for name, make, eps_list in cases:
        keys = make()
        torch.cuda.synchronize()
        n, kb = keys.numel(), keys.element_size()
        out = torch.empty_like(keys)
        # point queries on every variant's blob: 1e6 access(i), 1e6 lower_bound(q)
        nq = 1_000_000
        idx = workloads.uniform_indices(nq, n, seed=workloads.SEED_BASE + 107, device=dev)
        lo_k, hi_k = int(keys[0]) & ((1 << (8 * kb)) - 1), int(keys[-1]) & ((1 << (8 * kb)) - 1)
        qs = workloads.uniform_keys(nq, lo_k, hi_k, seed=workloads.SEED_BASE + 108, device=dev, key_bytes=kb)
        want_acc = keys[idx]
        if kb == 4:  # u32 bit patterns in int32: compare as unsigned
            want_pos = torch.searchsorted(keys.to(torch.int64) & 0xFFFFFFFF, qs.to(torch.int64) & 0xFFFFFFFF,
                                          side="left")
        else:
            want_pos = torch.searchsorted(keys, qs, side="left")
        acc = torch.empty_like(want_acc)
        pos = torch.empty(nq, dtype=torch.int64, device=dev)
        rows = {}
        for eps in eps_list:
            bmax, ws_bytes = lc.compress_bound(n, kb, eps, frac_bits=20, fit="opt")  # the largest of the variants
            blob = torch.empty(bmax, dtype=torch.uint8, device=dev)
            ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
            nb = torch.zeros(1, dtype=torch.int64, device=dev)
            fl = torch.zeros(1, dtype=torch.int32, device=dev)
            row = {}
            for label, fit, F in variants:
                lc.compress_async(keys, eps, blob, ws, nb, fl, frac_bits=F, fit=fit)
                torch.cuda.synchronize()
                marks = []
                for _ in range(reps):
                    e0, e1 = ev(), ev()
                    e0.record()
                    lc.compress_async(keys, eps, blob, ws, nb, fl, frac_bits=F, fit=fit)
                    e1.record()
                    marks.append((e0, e1))
                torch.cuda.synchronize()
                assert int(fl.item()) == 0, (name, eps, label, int(fl.item()))
                ms = float(np.mean([a.elapsed_time(b) for a, b in marks]))
                b = lc.Blob.from_device(blob)
                lc.decompress(b, out=out)
                torch.cuda.synchronize()
                assert torch.equal(out, keys), (name, eps, label, "round trip")
                dmarks = []
                for _ in range(reps):
                    e0, e1 = ev(), ev()
                    e0.record()
                    lc.decompress(b, out=out)
                    e1.record()
                    dmarks.append((e0, e1))
                torch.cuda.synchronize()
                dms = float(np.mean([a.elapsed_time(c) for a, c in dmarks]))
                lc.access(b, idx, out=acc, flags=fl, check=False)
                lc.lower_bound(b, qs, out=pos)
                torch.cuda.synchronize()
                assert int(fl.item()) == 0 and torch.equal(acc, want_acc) and torch.equal(pos, want_pos), \
                    (name, eps, label, "lookups")
                qmarks = []
                for _ in range(reps):
                    e0, e1, e2 = ev(), ev(), ev()
                    e0.record()
                    lc.access(b, idx, out=acc, flags=fl, check=False)
                    e1.record()
                    lc.lower_bound(b, qs, out=pos)
                    e2.record()
                    qmarks.append((e0, e1, e2))
                torch.cuda.synchronize()
                ams = float(np.mean([a.elapsed_time(c) for a, c, _ in qmarks]))
                lms = float(np.mean([c.elapsed_time(d) for _, c, d in qmarks]))
                row[label] = {"compress_ms": round(ms, 3), "keys_per_s": round(n / ms * 1e3, 1),
                              "decompress_ms": round(dms, 3), "decoded_GBps": round(n * kb / dms / 1e6, 1),
                              "access_lookups_per_s": round(nq / ams * 1e3, 1),
                              "lower_bound_lookups_per_s": round(nq / lms * 1e3, 1),
                              "bits_per_key": round(b.bits_per_key, 4), "nseg_total": b.info.nseg_total}
            g = row["greedy"]
            for label in ("min", "opt", "greedy_F0", "opt_F0"):
                row[label]["bytes_saved_pct_vs_greedy"] = round(100 * (1 - row[label]["bits_per_key"] / g["bits_per_key"]), 3)
                row[label]["segments_saved_pct_vs_greedy"] = round(100 * (1 - row[label]["nseg_total"] / g["nseg_total"]), 3)
            row["opt_F0"]["bytes_saved_pct_vs_greedy_F0"] = round(
                100 * (1 - row["opt_F0"]["bits_per_key"] / row["greedy_F0"]["bits_per_key"]), 3)
            rows[str(eps)] = row
            log(f"fits {name} eps={eps}: " + ", ".join(f"{k} {v['bits_per_key']} b/key {v['compress_ms']} ms"
                                                       for k, v in row.items()))
            del blob, ws
        res[name] = {"n": n, "key_bytes": kb, "per_eps": rows}
        del keys, out, idx, qs, want_acc, want_pos, acc, pos
        torch.cuda.empty_cache()
    return res


def _pick(d, keys):
    return {k: d[k] for k in keys if isinstance(d, dict) and k in d}


def headline(result: dict) -> dict:
    """The compact headline record printed last on stdout: the metric, the
    roofline of the dominant kernel (cold and warm), the CPU baseline and a
    few figures of each sub-measurement.  Everything else stays in the full
    record (stderr and the --full-json file)."""
    h = _pick(result, ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                       "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "roofline_warm"))
    enc = result.get("roofline_encode")
    if enc:
        h["roofline_encode"] = dict(_pick(enc, ("bound", "achieved", "peak", "unit", "frac", "avg_call_ms")),
                                    hbm_frac=enc.get("hbm", {}).get("frac"))
    cpu = result.get("cpu_baseline")
    if cpu:
        h["cpu_baseline"] = dict(_pick(cpu, ("value", "unit", "cores", "kind", "sample", "single_core_GBps")),
                                 host_cpu=cpu.get("host", {}).get("cpu"))
    pe = result.get("per_eps", {})
    h["ratio"] = {e: v.get("ratio") for e, v in pe.items()}
    h["compress_ms"] = {e: v.get("compress_ms") for e, v in pe.items()}
    h.update(_pick(result, ("decompress_range_GBps", "access_lookups_per_s", "lower_bound_lookups_per_s")))
    bt = result.get("batching")
    if bt:
        st = bt.get("step_ms", {})
        h["batching"] = {"decoded_GBps": bt.get("decoded_GBps"), "bits_per_key": bt.get("bits_per_key"),
                         "step_ms": _pick(st, ("batched_graph", "per_list_eager"))}
    sv = result.get("serving")
    if sv and sv.get("points"):
        h["serving"] = {"sat": _pick(sv["points"][-1], ("qps_achieved", "p50_us", "p99_us")),
                        "speedup_vs_unbatched": sv.get("saturation_speedup_vs_unbatched")}
    # drop the optional parts, least important first, until the line fits
    for k in ("compress_ms", "ratio", "serving", "batching"):
        if len(json.dumps(h)) <= HEADLINE_MAX_BYTES:
            break
        h.pop(k, None)
    if len(json.dumps(h)) > HEADLINE_MAX_BYTES and "cpu_baseline" in h:
        h["cpu_baseline"].pop("sample", None)
    return h


def emit(result: dict, full_json: str | None):
    """Full record to stderr (and to full_json when given), then the
    headline as the last line on stdout."""
    full = json.dumps(result)
    print(f"[bench] full record: {full}", file=sys.stderr, flush=True)
    if full_json:
        d = os.path.dirname(os.path.abspath(full_json))
        os.makedirs(d, exist_ok=True)
        with open(full_json, "w") as f:
            f.write(full + "\n")
    print(json.dumps(headline(result)), flush=True)


def _counter_rows(d: str):
    """(dispatch id, kernel name, counter name, value) of a rocprofv3 --pmc
    csv output folder, in dispatch order."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])))
    rows.sort()
    return rows


def summarize_traffic(fetch_dir: str, write_dir: str, n: int, eps_list, out: str = TRAFFIC_FILE):
    """profiles/decode_traffic.json from two counter runs (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch) of the core benchmark: both scaled by what
    they read for the untimed CALIB_COPY_BYTES copy; a decompress is cold
    when the dispatch before it is the FLUSH_BYTES flush copy, warm
    otherwise; decompress calls after the first (the untimed round-trip
    check) come in (warm, cold) pairs, one pair per eps in order."""
    import numpy as np
    def per_dispatch(d, counter):  # bytes per dispatch (rows of one dispatch summed)
        acc = {}
        for i, k, c, v in _counter_rows(d):
            if c == counter:
                acc[i] = (k, acc.get(i, (k, 0.0))[1] + v * 1024.0)
        return acc
    f, w = per_dispatch(fetch_dir, "FETCH_SIZE"), per_dispatch(write_dir, "WRITE_SIZE")
    if not f or not w:
        raise SystemExit(f"no FETCH_SIZE / WRITE_SIZE rows under {fetch_dir} / {write_dir}")
    copies = [i for i in sorted(w) if "decode" not in w[i][0]]
    calib = next(i for i in copies if abs(w[i][1] - CALIB_COPY_BYTES) < 0.05 * CALIB_COPY_BYTES)
    fs, ws = CALIB_COPY_BYTES / f[calib][1], CALIB_COPY_BYTES / w[calib][1]
    flush = {i for i in copies if abs(w[i][1] * ws - FLUSH_BYTES) < 0.05 * FLUSH_BYTES}
    dec = [i for i in sorted(w) if "decode_full_kernel<8, false>" in w[i][0]]
    by = {"cold": {str(e): [] for e in eps_list}, "warm": {str(e): [] for e in eps_list}}
    order = sorted(w)
    for k, i in enumerate(dec[1:]):
        prev = order[order.index(i) - 1]
        kind = "cold" if prev in flush else "warm"
        e = str(eps_list[(k // 2) % len(eps_list)])
        by[kind][e].append(f[i][1] * fs + w[i][1] * ws)
    rec = {"n": n, "eps": list(eps_list), "frac_bits": FRAC_BITS, "fetch_scale": round(fs, 4),
           "write_scale": round(ws, 4), "kernel_src_sha256_16": kernel_src_hash(),
           "kernels": ["decode_full_kernel<8, false>"]}
    for kind in ("cold", "warm"):
        vals = [v for e in by[kind] for v in by[kind][e]]
        rec[f"bytes_per_decompress_{kind}"] = int(np.mean(vals))
        rec[f"bytes_per_decompress_{kind}_by_eps"] = {e: int(np.mean(v)) for e, v in by[kind].items() if v}
        rec[f"calls_{kind}"] = len(vals)
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def summarize_valu(valu_dir: str, n: int, eps_list, out: str = VALU_FILE):
    """profiles/compress_valu.json from a counter run (SQ_INSTS_VALU) of the
    core benchmark restricted to the compress kernels: every lc_compress call
    starts with its fit kernel; calls come one per eps in order."""
    import numpy as np
    acc = {}
    for i, k, c, v in _counter_rows(valu_dir):
        if c == "SQ_INSTS_VALU":
            acc[i] = (k, acc.get(i, (k, 0.0))[1] + v)
    rows = [(i, k, v) for i, (k, v) in sorted(acc.items())]
    if not rows:
        raise SystemExit(f"no SQ_INSTS_VALU rows under {valu_dir}")
    calls, names = [], set()
    for i, k, v in rows:
        name = k.replace("void ", "").replace("lc::(anonymous namespace)::", "").split("(")[0]
        names.add(name)
        if "fit_" in name or not calls:
            calls.append(0.0)
        calls[-1] += v
    per = {str(e): [] for e in eps_list}
    for k, v in enumerate(calls):
        per[str(eps_list[k % len(eps_list)])].append(v)
    rec = {"n": n, "eps": list(eps_list), "frac_bits": FRAC_BITS,
           "valu_insts_per_call": {e: int(np.mean(v)) for e, v in per.items() if v},
           "calls_counted": {e: len(v) for e, v in per.items()},
           "kernel_src_sha256_16": kernel_src_hash(), "kernels": sorted(names)}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def main():
    global FRAC_BITS
    if len(sys.argv) > 1 and sys.argv[1] in ("--summarize-traffic", "--summarize-valu"):
        # host only: turn counter runs (rocprofv3 csv folders) into the profiles/*.json bench reads
        sp = argparse.ArgumentParser()
        sp.add_argument("dirs", nargs="+")
        sp.add_argument("--n", type=int, default=100_000_000)
        sp.add_argument("--eps", type=str, default="15,63,255")
        a = sp.parse_args(sys.argv[2:])
        eps_list = [int(e) for e in a.eps.split(",")]
        if sys.argv[1] == "--summarize-traffic":
            print(json.dumps(summarize_traffic(a.dirs[0], a.dirs[1], a.n, eps_list)))
        else:
            print(json.dumps(summarize_valu(a.dirs[0], a.n, eps_list)))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--eps", type=str, default="15,63,255")
    ap.add_argument("--access", type=int, default=10_000_000)
    ap.add_argument("--lower-bound", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--full-json", type=str, default="",
                    help="file that also receives the full result record (it always goes to stderr); "
                         "stdout's last line is the headline")
    ap.add_argument("--no-batch", action="store_true", help="skip the posting-list batch measurement")
    ap.add_argument("--batch-only", action="store_true", help="only the posting-list batch measurement")
    ap.add_argument("--no-serve", action="store_true", help="skip the request-server measurement")
    ap.add_argument("--serve-only", action="store_true", help="only the request-server measurement")
    ap.add_argument("--serve-n", type=int, default=1_000_000_000)
    ap.add_argument("--no-lookups", action="store_true", help="skip the heterogeneous-runs lookup measurement")
    ap.add_argument("--no-queries", action="store_true", help="skip the quantile / approximate / AND / OR measurement")
    ap.add_argument("--queries-only", action="store_true", help="only the quantile / approximate / AND / OR measurement")
    ap.add_argument("--frac-bits", type=int, default=FRAC_BITS,
                    help="fractional bits F of the slopes in every measured blob (the fit comparison sweeps its own)")
    ap.add_argument("--no-fits", action="store_true", help="skip the fit comparison (greedy, fewest anchored segments, optimal)")
    ap.add_argument("--fits-only", action="store_true", help="only the fit comparison (greedy, fewest anchored segments, optimal)")
    args = ap.parse_args()
    FRAC_BITS = args.frac_bits
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path is "
              "single-GPU here. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2412_10770_amd import lc, workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.batch_only:
        print(json.dumps(bench_batch(dev, args.steps, args.warmup)), flush=True)
        return
    if args.queries_only:
        print(json.dumps(bench_queries(dev)), flush=True)
        return
    if args.serve_only:
        print(json.dumps(bench_serve(dev, args.serve_n)), flush=True)
        return
    if args.fits_only:
        print(json.dumps(bench_fits(dev)), flush=True)
        return
    eps_list = [int(e) for e in args.eps.split(",")]
    t0 = time.perf_counter()
    keys = workloads.lognormal_distinct(args.n, device=dev)
    torch.cuda.synchronize()
    n = keys.numel()
    log(f"generated {n} keys in {time.perf_counter() - t0:.1f} s")

    # buffers (allocated once, outside the timed region)
    blobs, wss = {}, None
    max_ws = 0
    for e in eps_list:
        bmax, ws_bytes = lc.compress_bound(n, 8, e, frac_bits=FRAC_BITS)
        blobs[e] = torch.empty(bmax, dtype=torch.uint8, device=dev)
        max_ws = max(max_ws, ws_bytes)
    wss = torch.empty(max_ws, dtype=torch.uint8, device=dev)
    nbytes = torch.zeros(len(eps_list), dtype=torch.int64, device=dev)
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    out = torch.empty(n, dtype=torch.int64, device=dev)
    acc_idx = workloads.uniform_indices(args.access, n, seed=workloads.SEED_BASE + 102, device=dev)
    acc_out = torch.empty(args.access, dtype=torch.int64, device=dev)
    lo_k, hi_k = int(keys[0]), int(keys[-1])
    lb_q = workloads.uniform_keys(args.lower_bound, lo_k, hi_k, seed=workloads.SEED_BASE + 103, device=dev)
    lb_out = torch.empty(args.lower_bound, dtype=torch.int64, device=dev)
    r_begin, r_end = n // 4, n // 4 + n // 2
    r_out = torch.empty(r_end - r_begin, dtype=torch.int64, device=dev)

    # plain copy of known size: counter runs scale FETCH_SIZE / WRITE_SIZE by it
    calib_src = torch.ones(CALIB_COPY_BYTES // 8, dtype=torch.int64, device=dev)
    calib_dst = torch.empty_like(calib_src)
    calib_dst.copy_(calib_src)
    torch.cuda.synchronize()
    del calib_src, calib_dst
    # cache flush before every cold decode: a copy of FLUSH_BYTES (read and write) evicts the
    # blob from the 256 MB on-die cache and the L2s
    flush_src = torch.ones(FLUSH_BYTES // 8, dtype=torch.int64, device=dev)
    flush_dst = torch.empty_like(flush_src)

    # one untimed compress per eps to learn the blob layout (headers)
    infos = {}
    for k, e in enumerate(eps_list):
        lc.compress_async(keys, e, blobs[e], wss, nbytes[k:k + 1], flags, frac_bits=FRAC_BITS)
    torch.cuda.synchronize()
    assert int(flags.item()) == 0, "keys not sorted"
    for e in eps_list:
        infos[e] = lc.Blob.from_device(blobs[e])
    ref_eps = 63 if 63 in eps_list else eps_list[0]
    bref = infos[ref_eps]

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def step(timed: bool):
        """Per eps: compress, decompress at once (warm: the blob was just
        written), flush the caches, decompress again (cold); then the
        range, access and lower_bound batches on the eps = 63 blob."""
        rec = {}
        for k, e in enumerate(eps_list):
            b = lc.Blob(blobs[e], infos[e].info)
            e0, e1, e2, e3, e4 = ev(), ev(), ev(), ev(), ev()
            e0.record()
            lc.compress_async(keys, e, blobs[e], wss, nbytes[k:k + 1], flags, frac_bits=FRAC_BITS)
            e1.record()
            lc.decompress(b, out=out)
            e2.record()
            flush_dst.copy_(flush_src)
            e3.record()
            lc.decompress(b, out=out)
            e4.record()
            rec[e] = (e0, e1, e2, e3, e4)
        q0, q1, q2, q3 = ev(), ev(), ev(), ev()
        q0.record()
        lc.decompress_range(bref, r_begin, r_end, out=r_out)
        q1.record()
        lc.access(bref, acc_idx, out=acc_out, flags=flags, check=False)
        q2.record()
        lc.lower_bound(bref, lb_q, out=lb_out)
        q3.record()
        rec["q"] = (q0, q1, q2, q3)
        return rec

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    # correctness of the timed configuration: identity round trip
    lc.decompress(bref, out=out)
    torch.cuda.synchronize()
    assert torch.equal(out, keys), "round trip failed"
    log(f"warmup done ({args.warmup} steps); timing {args.steps} steps")

    recs = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        recs.append(step(True))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    log(f"timed region {wall:.3f} s")
    assert int(flags.item()) == 0
    del flush_src, flush_dst

    per_eps = {}
    alg_bytes = []
    cold_ms, warm_ms = [], []
    for e in eps_list:
        enc = [r[e][0].elapsed_time(r[e][1]) for r in recs]
        warm = [r[e][1].elapsed_time(r[e][2]) for r in recs]
        cold = [r[e][3].elapsed_time(r[e][4]) for r in recs]
        b = infos[e]
        cms, wms = float(np.mean(cold)), float(np.mean(warm))
        per_eps[str(e)] = {
            "ratio": round(b.ratio, 5), "bits_per_key": round(b.bits_per_key, 4),
            "blob_bytes": b.nbytes, "nseg_total": b.info.nseg_total,
            "paper_size_formula_bits_per_key": round((96 * b.info.nseg_total + n * b.info.width) / n, 4),
            "decode_ms_cold": round(cms, 4), "decode_GBps_cold": round(n * 8 / cms / 1e6, 2),
            "decode_ms_warm": round(wms, 4), "decode_GBps_warm": round(n * 8 / wms / 1e6, 2),
            "compress_ms": round(float(np.mean(enc)), 4),
            "compress_GBps": round(n * 8 / float(np.mean(enc)) / 1e6, 2),
        }
        cold_ms += cold
        warm_ms += warm
        alg_bytes.append(b.nbytes + n * 8)
    nd = len(cold_ms)
    value = n * 8 * nd / (sum(cold_ms) / 1e3) / 1e9
    value_warm = n * 8 * nd / (sum(warm_ms) / 1e3) / 1e9
    cold_avg, warm_avg = sum(cold_ms) / nd, sum(warm_ms) / nd
    bytes_per_launch = float(np.mean(alg_bytes))
    achieved = bytes_per_launch / (cold_avg / 1e3) / 1e9
    achieved_warm = bytes_per_launch / (warm_avg / 1e3) / 1e9
    rec = recorded_traffic()
    traffic = traffic_warm = None
    if rec is not None and rec.get("n") == n and rec.get("eps") == eps_list and rec.get("frac_bits") == FRAC_BITS:
        traffic = rec.get("bytes_per_decompress_cold")
        traffic_warm = rec.get("bytes_per_decompress_warm")
    # encode against both rooflines: HBM (keys read + blob written) and VALU
    # (issued lane-operations of the compress kernels, from the counter record)
    enc_ms = {e: float(np.mean([r[e][0].elapsed_time(r[e][1]) for r in recs])) for e in eps_list}
    enc_hbm = float(np.mean([(n * 8 + infos[e].nbytes) / (enc_ms[e] / 1e3) / 1e9 for e in eps_list]))
    vrec = recorded_valu()
    enc_alu = None
    if vrec is not None and vrec.get("n") == n and vrec.get("eps") == eps_list and vrec.get("frac_bits") == FRAC_BITS:
        enc_alu = float(np.mean([vrec["valu_insts_per_call"][str(e)] * 64 / (enc_ms[e] / 1e3) / 1e12
                                 for e in eps_list]))
    roofline_encode = {
        "bound": "alu", "kernel": "lc_compress (all its kernels)",
        "achieved": None if enc_alu is None else round(enc_alu, 2), "peak": round(VALU_PEAK_TOPS, 2),
        "unit": "T VALU lane-ops/s", "frac": None if enc_alu is None else round(enc_alu / VALU_PEAK_TOPS, 4),
        "traffic": None,
        "hbm": {"achieved": round(enc_hbm, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(enc_hbm / HBM_PEAK_GBPS, 4), "bytes": "8 n keys read + blob written"},
        "avg_call_ms": round(float(np.mean(list(enc_ms.values()))), 4),
        "valu_source": "profiles/compress_valu.json (rocprofv3 --pmc SQ_INSTS_VALU)" if enc_alu is not None
                       else "counter record absent or taken on other kernels",
    }
    rng_ms = float(np.mean([r["q"][0].elapsed_time(r["q"][1]) for r in recs]))
    acc_ms = float(np.mean([r["q"][1].elapsed_time(r["q"][2]) for r in recs]))
    lb_ms = float(np.mean([r["q"][2].elapsed_time(r["q"][3]) for r in recs]))

    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": f"{n} sorted distinct u64 keys, floor(2^40 x/M), x~lognormal(0,2); B=1024, F={FRAC_BITS}, "
                        f"eps {'/'.join(map(str, eps_list))}; per step and eps: compress, decode (warm), "
                        f"{FLUSH_BYTES >> 20} MiB flush copy, decode (cold: the value); then range of "
                        f"{r_end - r_begin} keys, {args.access} access, {args.lower_bound} lower_bound (eps {ref_eps})",
            "n": n, "key_bytes": 8, "log2_block": 10, "eps": eps_list, "frac_bits": FRAC_BITS,
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic, "cache": "cold",
            "kernel": "decode_full_kernel<8, false> (lc_decompress)",
            "bytes_per_launch": int(bytes_per_launch), "avg_launch_ms": round(cold_avg, 4),
        },
        "roofline_warm": {
            "bound": "hbm", "achieved": round(achieved_warm, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved_warm / HBM_PEAK_GBPS, 4), "traffic": traffic_warm, "cache": "warm",
            "avg_launch_ms": round(warm_avg, 4), "decoded_GBps": round(value_warm, 2),
        },
        "roofline_encode": roofline_encode,
        "per_eps": per_eps,
        "decompress_range_GBps": round((r_end - r_begin) * 8 / rng_ms / 1e6, 2),
        "access_lookups_per_s": round(args.access / acc_ms * 1e3, 1),
        "lower_bound_lookups_per_s": round(args.lower_bound / lb_ms * 1e3, 1),
        "paper_cpu_context": {"lc-simd": "6.535 GiB/s decode, Xeon Gold 6430, CCNews (Fig. 3a)"},
    }
    if not args.no_lookups:
        result["lookups"] = bench_lookups(dev)
        result["plain_method_1M"] = bench_small(dev)
        torch.cuda.empty_cache()
    if not args.no_queries:
        result["queries"] = bench_queries(dev)
        torch.cuda.empty_cache()
    if not args.no_fits:
        result["fits"] = bench_fits(dev, keys)
        torch.cuda.empty_cache()
    if not args.no_batch:
        del out, wss, blobs
        torch.cuda.empty_cache()
        result["batching"] = bench_batch(dev, args.steps, args.warmup)
        torch.cuda.empty_cache()
    if not args.no_serve:
        torch.cuda.empty_cache()
        result["serving"] = bench_serve(dev, args.serve_n)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a prefix of the keys")
        host = workloads.as_numpy(keys)
        result["cpu_baseline"] = cpu_baseline(host, eps_list)
    emit(result, args.full_json)


if __name__ == "__main__":
    main()
