"""Checks that pin the CPU oracle to facts fixed outside the oracle itself.

Each ``check_*`` takes a ``Ref`` (a build of the oracle) and raises
AssertionError when the build disagrees with:

* Def. 1 (lossless): decode(compress(K)) == K;
* Def. 2 (floor error bound): every key within eps of floor(f(i)), checked
  with Python integers from the segment list, and every stored code <= 2 eps,
  read back with a bit reader written here from the layout statement;
* Sec. II-A / Fig. 2: the residual width ceil(log2(2 eps + 1)) (eps = 4 gives
  4 bits in the paper's toy example);
* closed forms: an arithmetic progression fits one segment per block with
  every residual zero; the blob size from the segment counts;
* brute force on tiny inputs: every segment's slope is feasible, every
  segment that ends before its block does cannot be extended by one key with
  any slope, the stored slope is the midpoint of the enumerated feasible set,
  and the greedy count is at least the minimum over all anchored
  segmentations (equal when that minimum is 1);
* hand-derived worked examples under tests/golden/;
* the optimal fit (free fixed-point intercept): brute force over every
  integer (A, C) on tiny blocks for the greedy boundaries, the fewest
  segments over all segmentations, and the midpoint slope and intercept; a
  line with a fractional intercept is one segment at eps 0; the cap and the
  modulo-2^64 intercept at the top of the key range.

The same checks run against deliberately mutated builds of the oracle to
show that a plausible mistake in it fails at least one of them.
"""
from __future__ import annotations

import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def align16(x: int) -> int:
    return (x + 15) // 16 * 16


def widths_of(v: int) -> int:
    for nb in (1, 2, 4, 8):
        if v < (1 << (8 * nb)):
            return nb
    raise ValueError(v)


def load_golden(name: str) -> dict:
    out = {"blob": []}
    in_blob = False
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if in_blob:
                out["blob"].extend(int(t, 16) for t in line.split())
                continue
            key, _, val = line.partition(":")
            key, val = key.strip(), val.strip()
            if key == "blob":
                in_blob = True
            elif key == "keys":
                out["keys"] = [int(t) for t in val.split()]
            elif key == "fit":
                out["fit"] = val
            else:
                out[key] = int(val)
    out["blob"] = np.array(out["blob"], np.uint8)
    return out


def read_codes(blob: np.ndarray, h: dict, b: int, nb: int) -> list:
    """Codes of block b, read from the LSB-first bit stream of its slab."""
    w = h["width"]
    start = h["off_res"] + b * h["res_stride"]
    slab = int.from_bytes(bytes(blob[start:start + h["res_stride"]]), "little")
    mask = (1 << w) - 1
    return [(slab >> (j * w)) & mask for j in range(nb)]


# --- the random inputs the checks use ---------------------------------------

def _sorted_keys(rng, n, kb, kind):
    hi = (1 << (8 * kb)) - 1
    if kind == "uniform":
        g = rng.integers(0, 100, n)
    elif kind == "dups":
        g = rng.integers(0, 2, n)
    elif kind == "wide":
        g = rng.integers(0, 1 << min(20, 8 * kb - 14), n)
    else:  # bursty: long runs of small gaps with rare large jumps
        g = rng.integers(0, 5, n)
        jumps = rng.random(n) < 0.01
        g[jumps] = rng.integers(1000, 1 << min(24, 8 * kb - 14), int(jumps.sum()))
    k = np.cumsum(g.astype(np.uint64))
    room = hi - int(k[-1])  # keys may be shifted up by at most this much
    where = int(rng.integers(0, 3))
    if where == 0:
        base = 0
    elif where == 1:
        base = room  # the last key is the largest representable value
    else:
        base = int(rng.integers(0, min(room, 2 ** 62) + 1))
    return (k + np.uint64(base)).astype(np.uint32 if kb == 4 else np.uint64)


def random_cases(seed: int, count: int):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        kb = int(rng.choice([4, 8]))
        log2b = int(rng.integers(6, 13))
        n = int(rng.choice([1, 2, 63, 64, 65, 1000, 1 << log2b, (1 << log2b) + 1, 5000]))
        eps = int(rng.choice([0, 1, 3, 7, 15, 63, 255, 4095]))
        kind = str(rng.choice(["uniform", "dups", "wide", "bursty"]))
        yield _sorted_keys(rng, n, kb, kind), eps, log2b


# --- checks -------------------------------------------------------------------

def check_width(ref):
    assert ref.width(4) == 4, "Fig. 2: eps = 4 needs 4 bits"
    for eps, w in ((7, 4), (15, 5), (31, 6), (63, 7), (127, 8), (255, 9), (0, 0)):
        assert ref.width(eps) == w, (eps, w)
    for eps in list(range(0, 3000)) + [2 ** k + d for k in range(11, 31) for d in (-1, 0, 1)] + [2 ** 31 - 1]:
        assert ref.width(eps) == math.ceil(math.log2(2 * eps + 1)), eps


def check_roundtrip(ref, seed=1, count=60):
    for keys, eps, log2b in random_cases(seed, count):
        blob = ref.compress(keys, eps, log2b)
        back = ref.decode(blob)
        assert back.dtype == keys.dtype and np.array_equal(back, keys), (len(keys), eps, log2b)


def check_error_bound(ref, seed=2, count=40, frac_bits=20):
    for keys, eps, log2b in random_cases(seed, count):
        B = 1 << log2b
        blob = ref.compress(keys, eps, log2b, frac_bits)
        h = ref.header(blob)
        for b in range(0, (len(keys) + B - 1) // B):
            kk = [int(x) for x in keys[b * B:(b + 1) * B]]
            st, an, sl = ref.fit_block(np.array(kk, np.uint64), eps, frac_bits)
            assert int(st[0]) == 0
            for t in range(len(st)):
                s = int(st[t])
                e = int(st[t + 1]) if t + 1 < len(st) else len(kk)
                assert s < e and int(an[t]) == kk[s]
                for j in range(s, e):
                    pred = kk[s] + ((int(sl[t]) * (j - s)) >> frac_bits)
                    assert abs(kk[j] - pred) <= eps, (b, j, eps)
            codes = read_codes(blob, h, b, len(kk))
            assert max(codes) <= 2 * eps


def check_arithmetic_progression(ref, frac_bits=20):
    for g in (0, 1, 3, 64, 1000, 12345):
        for eps in (0, 7, 63, 5000):
            for log2b, kb in ((6, 4), (10, 8), (12, 8)):
                B = 1 << log2b
                n = 3 * B + 17
                keys = (np.uint64(11) + np.uint64(g) * np.arange(n, dtype=np.uint64))
                keys = keys.astype(np.uint32 if kb == 4 else np.uint64)
                blob = ref.compress(keys, eps, log2b, frac_bits)
                h = ref.header(blob)
                assert h["nseg_total"] == h["nblocks"], (g, eps, log2b)
                for b in range(h["nblocks"]):
                    nb = min(B, n - b * B)
                    assert read_codes(blob, h, b, nb) == [eps] * nb, (g, eps, b)
                _, _, sl = ref.fit_block(keys[:B].astype(np.uint64), eps, frac_bits)
                A = int(sl[0])
                # the midpoint lies in [g 2^F, g 2^F + 2^F / (B - 1)), so floor(A d / 2^F) = g d
                assert g * 2 ** frac_bits <= A and (A - g * 2 ** frac_bits) * (B - 1) < 2 ** frac_bits, (g, eps, A)


def check_span_within_eps(ref):
    rng = np.random.default_rng(5)
    for eps in (3, 63, 1000):
        for _ in range(20):
            k = np.sort(rng.integers(0, eps + 1, 500)).astype(np.uint64) + np.uint64(77)
            st, _, _ = ref.fit_block(k, eps)
            assert len(st) == 1, "a block whose key span is <= eps is one segment"


def _feasible_masks(kk, s, eps, F, alo, ahi):
    """For e = s+1 .. n: boolean mask over the integers A in [alo, ahi] of
    slopes keeping keys s..e-1 within eps (Def. 2), by enumeration."""
    A = np.arange(alo, ahi + 1, dtype=np.int64)
    mask = np.ones(len(A), bool)
    out = {s + 1: mask.copy()}
    for j in range(s + 1, len(kk)):
        pred = kk[s] + ((A * (j - s)) >> F)  # arithmetic shift: floor, also for A < 0
        mask &= np.abs(kk[j] - pred) <= eps
        out[j + 1] = mask.copy()
    return A, out


def check_bruteforce(ref, seed=3, trials=150):
    rng = np.random.default_rng(seed)
    greedy_above_min = 0
    for trial in range(trials):
        F = int(rng.choice([0, 1, 2, 4]))
        eps = int(rng.integers(0, 4))
        n = int(rng.integers(1, 13))
        kk = [int(x) for x in np.cumsum(rng.integers(0, int(rng.choice([3, 8, 20])), n))]
        alo, ahi = -((eps + 2) << F), (max(kk) - min(kk) + eps + 2) << F
        masks = {}
        for s in range(n):
            Avals, masks[s] = _feasible_masks(kk, s, eps, F, alo, ahi)
        nonneg = Avals >= 0

        st, an, sl = ref.fit_block(np.array(kk, np.uint64), eps, F)
        bounds = [int(x) for x in st] + [n]
        assert bounds[0] == 0 and all(a < b for a, b in zip(bounds, bounds[1:]))
        for t in range(len(st)):
            s, e, A = bounds[t], bounds[t + 1], int(sl[t])
            assert int(an[t]) == kk[s]
            if e - s == 1:
                assert A == 0
            else:
                feas = Avals[masks[s][e]]
                assert len(feas) and alo < feas[0] and feas[-1] < ahi, "enumeration range too small"
                assert np.array_equal(feas, np.arange(feas[0], feas[-1] + 1)), "feasible set is an interval"
                assert A == max(0, (int(feas[0]) + int(feas[-1])) // 2), (kk, eps, F, s, e, A)
                assert (masks[s][e] & nonneg).any(), "the segment must admit a slope >= 0"
            if e < n:
                assert not (masks[s][e + 1] & nonneg).any(), ("segment could be extended", kk, eps, F, s, e)

        # minimum number of anchored segments with slopes >= 0, by dynamic programming
        INF = 10 ** 9
        dp = [0] + [INF] * n
        for e in range(1, n + 1):
            for s in range(e):
                if (masks[s][e] & nonneg).any():
                    dp[e] = min(dp[e], dp[s] + 1)
        assert len(st) >= dp[n]
        if dp[n] == 1:
            assert len(st) == 1
        greedy_above_min += len(st) > dp[n]
    return greedy_above_min


def check_cap_boundary(ref, frac_bits=20):
    cap = 1 << (64 - frac_bits)
    for eps in (0, 5):
        joined = np.array([0, cap - 2 - eps], np.uint64)  # D + eps + 1 = cap - 1
        split = np.array([0, cap - 1 - eps], np.uint64)   # D + eps + 1 = cap
        assert len(ref.fit_block(joined, eps, frac_bits)[0]) == 1
        assert len(ref.fit_block(split, eps, frac_bits)[0]) == 2
    huge = np.cumsum(np.full(300, 1 << 45, dtype=np.uint64))
    st, _, sl = ref.fit_block(huge, 3, frac_bits)
    assert len(st) == 300 and not sl.any()
    assert np.array_equal(ref.decode(ref.compress(huge, 3, 8, frac_bits)), huge)


def check_blob_size(ref, seed=4, count=30):
    for keys, eps, log2b in random_cases(seed, count):
        B = 1 << log2b
        kb = keys.dtype.itemsize
        w = math.ceil(math.log2(2 * eps + 1))
        nblocks = (len(keys) + B - 1) // B
        stride = align16((B * w + 7) // 8)
        size = 128 + align16(nblocks * kb) + 16 * nblocks + nblocks * stride
        nseg_total = 0
        for b in range(nblocks):
            kk = keys[b * B:(b + 1) * B].astype(np.uint64)
            st, an, sl = ref.fit_block(kk, eps)
            m = len(st)
            nseg_total += m
            ab = widths_of(int(an.max() - an[0]))
            sb = widths_of(int(sl.max()))
            size += align16(2 * m) + align16(ab * m) + align16(sb * m)
        blob = ref.compress(keys, eps, log2b)
        h = ref.header(blob)
        assert len(blob) == size == h["blob_bytes"]
        assert h["nseg_total"] == nseg_total and h["nblocks"] == nblocks and h["n"] == len(keys)
        assert h["off_dir"] == 128 + align16(nblocks * kb)
        assert h["off_res"] == h["off_dir"] + 16 * nblocks and h["res_stride"] == stride


def check_byte_widths(ref):
    # anchor deltas 255 / 256 and 65535 / 65536 sit on either side of a width step
    for delta, ab in ((255, 1), (256, 2), (65535, 2), (65536, 4), (2 ** 32 - 1, 4), (2 ** 32, 8)):
        keys = np.array([0, 0, delta], np.uint64)  # eps 0: the jump starts a new segment
        blob = ref.compress(keys, 0, 6)
        h = ref.header(blob)
        assert h["nseg_total"] == 2
        assert int(blob[h["off_dir"] + 14]) == ab, (delta, ab)


def check_golden(ref):
    for name in ("ap4_eps1.txt", "break4_eps1.txt", "opt4_frac_eps0.txt"):
        g = load_golden(name)
        keys = np.array(g["keys"], np.uint32 if g["key_bytes"] == 4 else np.uint64)
        blob = ref.compress(keys, g["eps"], g["log2_block"], g["frac_bits"], fit=g.get("fit", "greedy"))
        assert np.array_equal(blob, g["blob"]), name
        assert np.array_equal(ref.decode(g["blob"]), keys), name


ALL_CHECKS = [check_width, check_golden, check_roundtrip, check_error_bound,
              check_arithmetic_progression, check_span_within_eps, check_bruteforce,
              check_cap_boundary, check_blob_size, check_byte_widths]


# --- fewest-segment fit ---------------------------------------------------------

def feasible_slopes(k, s, e, eps, F):
    """All integer A (any sign) with |K[i] - (K[s] + floor(A (i - s) / 2^F))|
    <= eps for s < i < e, by trying every A that could qualify: for d >= 1 a
    slope with |A| > (span + eps + 1) 2^F predicts outside [K[s] - span - eps,
    K[s] + span + eps] already at d = 1."""
    span = int(k[e - 1]) - int(k[s])
    amax = (span + eps + 1) << F
    return [A for A in range(-amax, amax + 1)
            if all(abs(int(k[i]) - (int(k[s]) + ((A * (i - s)) >> F))) <= eps for i in range(s + 1, e))]


def brute_min_segmentations(k, eps, F):
    """(fewest segments, componentwise-earliest boundaries of the minimum
    segmentations) over every segmentation of k into feasible segments."""
    n = len(k)
    ok = {(s, e): bool(feasible_slopes(k, s, e, eps, F)) for s in range(n) for e in range(s + 1, n + 1)}
    best, optimal = None, []
    for mask in range(1 << max(n - 1, 0)):  # a cut after key i when bit i is set
        cuts = [0] + [i + 1 for i in range(n - 1) if (mask >> i) & 1] + [n]
        if all(ok[(a, b)] for a, b in zip(cuts, cuts[1:])):
            m = len(cuts) - 1
            if best is None or m < best:
                best, optimal = m, [cuts]
            elif m == best:
                optimal.append(cuts)
    return best, [min(c[j] for c in optimal) for j in range(best + 1)]


def expected_slope(k, s, e, eps, F):
    """The midpoint rule on the brute-force interval of feasible slopes."""
    if e - s == 1:
        return 0
    sl = feasible_slopes(k, s, e, eps, F)
    lo, hi = min(sl), max(sl)
    assert sl == list(range(lo, hi + 1))  # the feasible slopes form an interval
    return max(0, (lo + hi) // 2)


def check_min_fit_bruteforce(ref, trials=800, seed=11):
    """fit="min": the fewest segments, the earliest boundaries among the
    minimum segmentations, and the midpoint slope of each segment, all by
    brute force on tiny blocks; the trials must include blocks where the
    greedy fit is not minimal."""
    rng = np.random.default_rng(seed)
    greedy_worse = 0
    for trial in range(trials):
        n = int(rng.integers(1, 9))
        eps = int(rng.integers(0, 4))
        F = int(rng.choice([0, 1, 3]))
        hi = int(rng.choice([8, 24, 60]))
        k = np.sort(rng.integers(0, hi, n)).astype(np.uint64)
        st, an, sl = ref.fit_block(k, eps, F, "min")
        best, earliest = brute_min_segmentations(k, eps, F)
        assert len(st) == best, (trial, k.tolist(), eps, F)
        assert st.tolist() == earliest[:-1], (trial, k.tolist(), eps, F)
        ends = st.tolist()[1:] + [n]
        for s, e, a, A in zip(st.tolist(), ends, an.tolist(), sl.tolist()):
            assert a == int(k[s])
            assert A == expected_slope(k, s, e, eps, F), (trial, k.tolist(), eps, F, s, e)
        greedy_worse += len(ref.fit_block(k, eps, F)[0]) > best
    assert greedy_worse > 0


def check_min_fit_blobs(ref, seed=1, count=10):
    """fit="min" blobs decode, and never hold more segments than greedy ones."""
    for keys, eps, log2b in random_cases(seed, count):
        keys = keys[:20000]
        for F in (0, 20):
            g = ref.compress(keys, eps, log2b, F)
            m = ref.compress(keys, eps, log2b, F, fit="min")
            assert ref.header(m)["nseg_total"] <= ref.header(g)["nseg_total"]
            assert np.array_equal(ref.decode(m), keys)


# --- optimal fit: free fixed-point intercept ---------------------------------------

def opt_lines(k, s, e, eps, F, first):
    """Boolean grid over (A, C) of the lines floor((C + A d) / 2^F) that keep
    keys s .. e-1 within eps, with A >= 0 and C >= first 2^F, tried by
    evaluating the floor for every key (numpy int64; tiny keys and F only).
    Returns (A values, C values, mask)."""
    ks = [int(x) for x in k]
    span = ks[e - 1] - ks[s]
    A = np.arange(0, ((span + 2 * eps + 1) << F) + 1, dtype=np.int64)
    # key s alone: K[s] - eps <= floor(C / 2^F) <= K[s] + eps
    c_lo = max((ks[s] - eps) << F, first << F)
    C = np.arange(c_lo, ((ks[s] + eps + 1) << F), dtype=np.int64)
    ok = np.ones((len(A), len(C)), bool)
    for i in range(s, e):
        pred = (C[None, :] + A[:, None] * (i - s)) >> F
        ok &= np.abs(ks[i] - pred) <= eps
    return A, C, ok


def opt_feasible(k, s, e, eps, F, first):
    if ((int(k[e - 1]) - int(k[s]) + 2 * eps + 1) >> (64 - F)) != 0:  # the cap
        return False
    return bool(opt_lines(k, s, e, eps, F, first)[2].any())


def check_opt_fit_bruteforce(ref, trials=300, seed=12):
    """fit="opt" on tiny blocks against the grid: each segment is the longest
    feasible one from its start, their number is the minimum over every
    segmentation, and the stored A and C are the midpoints of the feasible
    slopes and of that slope's feasible intercepts.  The trials must include
    blocks where the anchored minimum needs more segments."""
    rng = np.random.default_rng(seed)
    beats_anchored = 0
    for trial in range(trials):
        n = int(rng.integers(1, 8))
        eps = int(rng.integers(0, 3))
        F = int(rng.choice([0, 1, 2]))
        hi = int(rng.choice([6, 20, 40]))
        k = np.sort(rng.integers(0, hi, n)).astype(np.uint64)
        first = int(k[0])
        st, an, sl, fr = ref.fit_block(k, eps, F, "opt")
        ok = {(a, b): opt_feasible(k, a, b, eps, F, first) for a in range(n) for b in range(a + 1, n + 1)}
        ends = st.tolist()[1:] + [n]
        for s_, e_ in zip(st.tolist(), ends):
            assert ok[(s_, e_)], (trial, k.tolist(), eps, F, s_, e_)
            assert e_ == n or not ok[(s_, e_ + 1)], (trial, k.tolist(), eps, F, s_, e_)
        # fewest segments over every segmentation (dynamic programming)
        best = [0] + [n + 1] * n
        for b in range(1, n + 1):
            best[b] = min(best[a] + 1 for a in range(b) if ok[(a, b)])
        assert len(st) == best[n], (trial, k.tolist(), eps, F)
        for s_, e_, a, A_, c in zip(st.tolist(), ends, an.tolist(), sl.tolist(), fr.tolist()):
            As, Cs, m = opt_lines(k, s_, e_, eps, F, first)
            feas_A = As[m.any(axis=1)].tolist()
            assert feas_A == list(range(feas_A[0], feas_A[-1] + 1))  # an interval
            want_A = 0 if e_ - s_ == 1 else (feas_A[0] + feas_A[-1]) // 2
            assert A_ == want_A, (trial, k.tolist(), eps, F, s_, e_)
            feas_C = Cs[m[want_A - int(As[0])]].tolist()
            assert feas_C == list(range(feas_C[0], feas_C[-1] + 1))
            want_C = (feas_C[0] + feas_C[-1]) // 2
            assert (int(a) << F) + int(c) == want_C and int(c) < (1 << F), (trial, k.tolist(), eps, F, s_)
        beats_anchored += len(ref.fit_block(k, eps, F, "min")[0]) > len(st)
    assert beats_anchored > 0


def check_opt_fit_closed_forms(ref):
    """A fixed-point line with a fractional intercept is one segment at eps 0
    (the anchored fits need more), rebuilt exactly; the cap
    K[e] - K[s] + 2 eps + 1 < 2^(64 - F) at its boundary; intercepts past
    2^64 near the top of the key range decode modulo 2^64."""
    for F, A0, C0 in ((8, 700, 5 * 256 + 200), (20, 3 << 19, 77), (0, 3, 11)):
        k = np.array([(C0 + A0 * i) >> F for i in range(512)], np.uint64)
        st, an, sl, fr = ref.fit_block(k, 0, F, "opt")
        assert len(st) == 1
        pred = [((int(an[0]) << F) + int(fr[0]) + int(sl[0]) * i) >> F for i in range(512)]
        assert pred == k.tolist()
        if F == 8:
            assert len(ref.fit_block(k, 0, F, "min")[0]) > 1
        blob = ref.compress(k, 0, 9, F, fit="opt")
        assert np.array_equal(ref.decode(blob), k)
    for F in (20, 32):
        cap = 1 << (64 - F)
        for eps in (0, 5):
            joined = np.array([0, cap - 2 - 2 * eps], np.uint64)  # K[1] - K[0] + 2 eps + 1 = cap - 1
            split = np.array([0, cap - 1 - 2 * eps], np.uint64)   # ... = cap
            assert len(ref.fit_block(joined, eps, F, "opt")[0]) == 1
            assert len(ref.fit_block(split, eps, F, "opt")[0]) == 2
            for kk in (joined, split):
                assert np.array_equal(ref.decode(ref.compress(kk, eps, 6, F, fit="opt")), kk)
    top = (1 << 64) - 1
    for eps in (3, 100):
        k = np.array(sorted({0, 9, top - 300, top - 40, top - 3, top - 1, top}), np.uint64)
        for F in (0, 20):
            blob = ref.compress(k, eps, 6, F, fit="opt")
            assert np.array_equal(ref.decode(blob), k)
            h = ref.header(blob)
            assert h["flags"] == 1 and h["nseg_total"] <= len(ref.fit_block(k, eps, F, "min")[0])


def check_opt_fit_blobs(ref, seed=5, count=8):
    """fit="opt" blobs decode (4- and 8-byte keys, F from 0 to 32), keep
    every prediction within eps, never hold more segments than the anchored
    minimum, and have the size the layout statement gives: the fraction
    array takes 0, 1, 2 or 4 bytes per segment for F = 0, <= 8, <= 16, more."""
    for keys, eps, log2b in random_cases(seed, count):
        keys = keys[:6000]
        for F in (0, 5, 12, 20, 32):
            m = ref.compress(keys, eps, log2b, F, fit="min")
            o = ref.compress(keys, eps, log2b, F, fit="opt")
            ho = ref.header(o)
            assert ho["flags"] == 1 and ref.header(m)["flags"] == 0
            assert ho["nseg_total"] <= ref.header(m)["nseg_total"]
            assert np.array_equal(ref.decode(o), keys)
            fb = 0 if F == 0 else 1 if F <= 8 else 2 if F <= 16 else 4
            B = 1 << log2b
            size = ho["off_seg"]
            for b0 in range(0, len(keys), B):
                st, an, sl, fr = ref.fit_block(keys[b0:b0 + B], eps, F, "opt")
                nseg = len(st)
                first = int(keys[b0])
                dmax = max(((int(a) - first) % (1 << 64)) for a in an)
                size += (align16(2 * nseg) + align16(widths_of(dmax) * nseg) +
                         align16(widths_of(int(sl.max())) * nseg) + align16(fb * nseg))
                ends = st.tolist()[1:] + [min(B, len(keys) - b0)]
                for s_, e_, a, A_, c in zip(st.tolist(), ends, an.tolist(), sl.tolist(), fr.tolist()):
                    for j in range(s_, e_):
                        f = (int(a) + ((int(A_) * (j - s_) + int(c)) >> F)) % (1 << 64)
                        d = (int(keys[b0 + j]) - f + (1 << 63)) % (1 << 64) - (1 << 63)
                        assert abs(d) <= eps
            assert size == ho["blob_bytes"] == len(o)


def run_quick(ref) -> str:
    """Run every check with small counts; return the name of the first that fails, or ''."""
    quick = [
        (check_width, {}), (check_golden, {}), (check_roundtrip, {"count": 25}),
        (check_error_bound, {"count": 12}), (check_arithmetic_progression, {}),
        (check_span_within_eps, {}), (check_bruteforce, {"trials": 200}),
        (check_cap_boundary, {}), (check_blob_size, {"count": 12}), (check_byte_widths, {}),
        (check_min_fit_bruteforce, {"trials": 400}), (check_min_fit_blobs, {"count": 6}),
        (check_opt_fit_closed_forms, {}), (check_opt_fit_bruteforce, {"trials": 150}),
        (check_opt_fit_blobs, {"count": 8}),
    ]
    for fn, kw in quick:
        try:
            fn(ref, **kw)
        except Exception:  # an assertion, an oracle error status, or a malformed result
            return fn.__name__
    return ""
