/*
 * lcref.c -- CPU oracle for the learned integer compressor.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or helper with the
 * HIP library: it reads and writes the blob format from its own statement of
 * it below.
 *
 * What it computes (paper: "Learned Data Compression: Challenges and
 * Opportunities for the Future", arXiv 2412.10770):
 *
 *   Def. 1 (Lossless Integer Compression): an encoding K^c of a sorted list K
 *   with Dec(K^c)[i] = K[i] for every i.
 *
 *   Def. 2 / Eq. 1 (eps-PLA): a piecewise linear f, segment j being
 *   (s_j, alpha_j, beta_j) with f(i) = alpha_j (i - s_j) + beta_j, such that
 *   |K[i] - floor(f(i))| <= eps for every i.
 *
 *   Sec. II-A: K^c = (f, Delta) with Delta[i] = K[i] - floor(f(i)) in
 *   [-eps, eps], each residual stored in ceil(log2(2 eps + 1)) bits, and
 *   decoding K[i] = floor(f(i)) + Delta[i].
 *
 * Readings taken where the paper is silent (each is listed in the design
 * notes of the repository):
 *   - slope alpha = A / 2^F with an integer A >= 0 (F fractional bits) and the
 *     intercept beta = K[s] (the segment is anchored at its first key), so
 *     floor(f(i)) = K[s] + floor(A (i - s) / 2^F) is exact integer arithmetic;
 *   - keys are split into fixed blocks of B = 2^log2_block keys and a segment
 *     never crosses a block boundary;
 *   - each segment is grown greedily key by key while some integer A keeps
 *     every key of the segment within eps (a shrinking cone of feasible A),
 *     with a cap that keeps A (i - s) below 2^64; the stored A is the midpoint
 *     of the final feasible interval of integer slopes (its lower end not
 *     clamped at zero), then clamped to A >= 0; A = 0 for a one-key segment;
 *   - the fewest-segment fit (fit = 1) keeps that class of segments and that
 *     slope rule and chooses the boundaries: a minimum number of segments per
 *     block, and of the minimum segmentations the one whose every boundary
 *     lies earliest (lcref_fit_block_min);
 *   - the optimal fit (fit = 2) widens the class to lines with a free
 *     fixed-point intercept, floor(f(i)) = floor((C + A (i - s)) / 2^F) with
 *     integers A >= 0 and C >= first_key 2^F (the line class of the optimal
 *     eps-PLA of Sec. II-A written in fixed point); a segment grows greedily
 *     while some (A, C) keeps every key within eps, which in this class gives
 *     the fewest segments (lcref_fit_block_opt);
 *   - a residual is stored offset by eps: code = Delta + eps in [0, 2 eps];
 *   - indices are 0-based.
 *
 * All cone arithmetic is done exactly in (signed) __int128 so that the
 * oracle does not depend on the overflow argument behind the cap.
 *
 * Blob v1 (little-endian, offsets in bytes from the blob start, every region
 * starting on a 16-byte boundary, every pad byte zero):
 *
 *   header, 128 bytes
 *      0 u32 magic 0x3142434C ("LCB1")   4 u16 version (1)
 *      6 u8  key_bytes (4|8)             7 u8  log2_block (6..12)
 *      8 u8  frac_bits F (0..32)         9 u8  width w
 *     10 u8  flags (bit 0: intercept fractions; no other bit is set)
 *     11 u8  0                          12 u32 eps
 *     16 u64 n                          24 u64 nblocks = ceil(n / B)
 *     32 u64 nseg_total                 40 u32 max_nseg (largest per block)
 *     44 u32 max_seg_bytes (largest segment area of a block)
 *                                       48 u64 off_first (= 128)
 *     56 u64 off_dir                    64 u64 off_res
 *     72 u64 res_stride                 80 u64 off_seg
 *     88 u64 blob_bytes                 96..127 zero
 *   first_keys[nblocks]   key_bytes each, region padded to 16
 *   dir[nblocks]          16 bytes each:
 *                           u64 seg_off (absolute), u32 nseg, u16 nkeys-1,
 *                           u8 anchor_bytes, u8 slope_bytes
 *   residual slabs        block b at off_res + b * res_stride,
 *                         res_stride = align16(ceil(B * w / 8)); code j of the
 *                         block occupies bits [j w, j w + w), bit p being bit
 *                         (p mod 8) of byte floor(p / 8) (LSB-first stream)
 *   segment areas         block by block in order, from off_seg:
 *                           u16 start[nseg]                padded to 16
 *                           anchor_delta[nseg] (K[s]-first_key[b]),
 *                                 anchor_bytes each         padded to 16
 *                           A[nseg], slope_bytes each      padded to 16
 *                           with flag bit 0 only (optimal fit):
 *                           frac[nseg], frac_bytes each    padded to 16
 *                           (frac_bytes = 0 if F = 0, 1 if F <= 8, 2 if
 *                           F <= 16, else 4: the array is absent at F = 0)
 *                         anchor_bytes / slope_bytes = the smallest of
 *                         1, 2, 4, 8 bytes holding the block's largest value.
 *   decoding key j of block b in segment t (d = j - start[t]):
 *     K = first_key[b] + anchor_delta[t] + floor((A[t] d + frac[t]) / 2^F)
 *         + code_j - eps  (mod 2^(8 key_bytes)), frac = 0 without the flag;
 *   with fractions, anchor_delta is floor(C / 2^F) - first_key[b] taken
 *   modulo 2^64 and frac = C mod 2^F.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define REF_OK 0
#define REF_EINVAL (-1)
#define REF_ENOSPC (-2)
#define REF_EFORMAT (-3)
#define REF_EUNSORTED (-5)

#define REF_MAGIC 0x3142434Cu
#define REF_VERSION 1u
#define REF_HEADER 128u
#define REF_FLAG_FRAC 1u

static uint64_t align16(uint64_t x) { return (x + 15u) / 16u * 16u; }

/* Bytes of one intercept fraction C mod 2^F: enough for F bits. */
static int frac_bytes(uint32_t F) { return F == 0 ? 0 : F <= 8 ? 1 : F <= 16 ? 2 : 4; }

/* Residual width: the smallest w with 2^w >= 2 eps + 1 (Sec. II-A). */
int lcref_width(uint32_t eps)
{
    uint64_t values = 2ull * (uint64_t)eps + 1ull;
    int w = 0;
    while ((1ull << w) < values)
        w++;
    return w;
}

/* Smallest of 1, 2, 4, 8 bytes that holds v. */
static int byte_width(uint64_t v)
{
    if (v < (1ull << 8)) return 1;
    if (v < (1ull << 16)) return 2;
    if (v < (1ull << 32)) return 4;
    return 8;
}

static uint64_t load_key(const void* keys, int kb, uint64_t i)
{
    if (kb == 4) return ((const uint32_t*)keys)[i];
    return ((const uint64_t*)keys)[i];
}

/*
 * Greedy anchored fit of one block (Def. 2 restricted to anchored segments
 * with integer fixed-point slope).  k[0..nb) are the block's keys.  For a
 * segment starting at s, a key e joins when some integer A satisfies
 *     K[e] - eps <= K[s] + floor(A d / 2^F) <= K[e] + eps,   d = e - s,
 * for it and every earlier key of the segment; with D = K[e] - K[s] that is
 *     ceil((D - eps) 2^F / d) <= A <= floor(((D + eps + 1) 2^F - 1) / d).
 * The segment stops at the first key for which the running intersection
 * [lo, hi] is empty, or whose D + eps + 1 reaches 2^(64 - F) (the cap).
 * The upper ends are never negative (keys are sorted), so the intersection
 * is non-empty exactly when it holds a non-negative A.  The stored slope is
 * the midpoint floor((lo + hi) / 2) of the final interval -- lo taken
 * without clamping at zero -- clamped to A >= 0; a one-key segment has A = 0.
 * Writes nseg segments (start, anchor, A); returns nseg.
 */
typedef __int128 i128;

/* The cone of the segment anchored at s, grown over candidates s+1 .. limit-1:
 * returns the end e (exclusive) of the longest feasible prefix (s < e <=
 * limit) and leaves its interval of integer slopes in [*lo, *hi]
 * (unbounded for a one-key segment). */
static uint32_t cone(const uint64_t* k, uint32_t s, uint32_t limit, uint32_t eps, uint32_t F, i128* lo,
                     i128* hi)
{
    const i128 scale = (i128)1 << F;
    const i128 cap = (i128)1 << (64 - F);
    const uint64_t anchor = k[s];
    i128 l_run = -((i128)1 << 100), h_run = (i128)1 << 100;
    uint32_t e = s + 1;
    while (e < limit) {
        i128 d = (i128)(e - s);
        i128 D = (i128)k[e] - (i128)anchor;
        if (D + eps + 1 >= cap)
            break;
        i128 num_lo = (D - eps) * scale;          /* may be negative */
        i128 l = num_lo >= 0 ? (num_lo + d - 1) / d : -((-num_lo) / d); /* ceil */
        i128 h = ((D + eps + 1) * scale - 1) / d; /* floor, never negative */
        i128 nlo = l_run > l ? l_run : l;
        i128 nhi = h_run < h ? h_run : h;
        if (nlo > nhi)
            break;
        l_run = nlo;
        h_run = nhi;
        e++;
    }
    *lo = l_run;
    *hi = h_run;
    return e;
}

/* Stored slope of the segment [s, e) with slope interval [lo, hi]. */
static uint64_t slope_of(uint32_t s, uint32_t e, i128 lo, i128 hi)
{
    if (e <= s + 1)
        return 0;
    i128 A = lo + (hi - lo) / 2; /* floor((lo + hi) / 2): hi - lo >= 0 */
    return A < 0 ? 0 : (uint64_t)A;
}

uint32_t lcref_fit_block(const uint64_t* k, uint32_t nb, uint32_t eps, uint32_t F,
                         uint32_t* seg_start, uint64_t* seg_anchor, uint64_t* seg_A)
{
    uint32_t nseg = 0;
    uint32_t s = 0;
    while (s < nb) {
        i128 lo, hi;
        uint32_t e = cone(k, s, nb, eps, F, &lo, &hi);
        seg_start[nseg] = s;
        seg_anchor[nseg] = k[s];
        seg_A[nseg] = slope_of(s, e, lo, hi);
        nseg++;
        s = e;
    }
    return nseg;
}

/*
 * Fewest segments within the same anchored class (the same segments the
 * greedy fit may form, chosen to minimise their number; Def. 2 with the
 * optimal-L goal of Sec. II-A restricted to anchored fixed-point segments).
 * reach[s] is the end of the greedy segment anchored at s: the segment [s, e)
 * is feasible exactly when e <= reach[s] (the cone only narrows as keys join).
 * Going backwards from the end of the block, every boundary is the smallest
 * s whose reach covers the boundary after it.  This gives a minimum number of
 * segments, and of all minimum segmentations the one whose every boundary
 * lies earliest: if c_0 < ... < c_m = nb is any feasible segmentation, then
 * induction from the end shows the chosen b_j <= c_j, so the chosen chain
 * reaches 0 within m steps.  Each segment's slope is then the midpoint rule
 * of the greedy fit applied to the cone of exactly that segment.
 */
uint32_t lcref_fit_block_min(const uint64_t* k, uint32_t nb, uint32_t eps, uint32_t F,
                             uint32_t* seg_start, uint64_t* seg_anchor, uint64_t* seg_A)
{
    if (nb == 0)
        return 0;
    uint32_t* reach = malloc(nb * sizeof(uint32_t));
    uint32_t* bound = malloc((nb + 1) * sizeof(uint32_t));
    if (!reach || !bound)
        abort(); /* a test oracle: fail loudly rather than return a wrong fit */
    for (uint32_t s = 0; s < nb; s++) {
        i128 lo, hi;
        reach[s] = cone(k, s, nb, eps, F, &lo, &hi);
    }
    /* boundaries from the end: bound[0] = nb, bound[1], ..., bound[m] = 0 */
    uint32_t m = 0;
    bound[0] = nb;
    while (bound[m] > 0) {
        uint32_t s = 0;
        while (reach[s] < bound[m]) /* s = bound[m] - 1 always qualifies */
            s++;
        bound[++m] = s;
    }
    for (uint32_t t = 0; t < m; t++) {
        uint32_t s = bound[m - t], e = bound[m - t - 1];
        i128 lo, hi;
        uint32_t got = cone(k, s, e, eps, F, &lo, &hi);
        (void)got; /* == e: [s, e) is feasible because e <= reach[s] */
        seg_start[t] = s;
        seg_anchor[t] = k[s];
        seg_A[t] = slope_of(s, e, lo, hi);
    }
    free(reach);
    free(bound);
    return m;
}

/* floor(a / b) and ceil(a / b) for b > 0 (C division truncates toward 0). */
static i128 floor_div(i128 a, i128 b)
{
    i128 q = a / b;
    if (a % b != 0 && a < 0)
        q--;
    return q;
}

static i128 ceil_div(i128 a, i128 b) { return -floor_div(-a, b); }

/*
 * Optimal fit (fit = 2): the class of fixed-point lines with a free intercept
 * (Def. 2 / Eq. 1 with any beta; the optimal eps-PLA of Sec. II-A, in fixed
 * point): floor(f(i)) = floor((C + A d) / 2^F), d = i - s, integers A >= 0
 * and C.  Key i of the segment is within eps exactly when
 *     Lo_i <= C + A d_i <= Up_i,
 *     Lo_i = (K[i] - eps) 2^F,   Up_i = (K[i] + eps + 1) 2^F - 1.
 * The blob keeps floor(C / 2^F) - first_key as the anchor delta, so C must
 * also be at least first_key 2^F: Lo_s is raised to max(K[s] - eps,
 * first_key) 2^F.  For an integer A, the feasible C are the integers of
 * [max_i (Lo_i - A d_i), min_i (Up_i - A d_i)]; that interval is non-empty
 * exactly when every pair i < j has Lo_j - Up_i <= A (j - i) <= Up_j - Lo_i.
 * So the feasible slopes are the integers of
 *     lo = max(0, max_{i<j} ceil((Lo_j - Up_i) / (j - i))),
 *     hi = min_{i<j} floor((Up_j - Lo_i) / (j - i)),
 * and a key e joins the segment when [lo, hi] stays non-empty with the pairs
 * (i, e) added and K[e] - K[s] + 2 eps + 1 < 2^(64 - F) (the cap, which keeps
 * A d + (C mod 2^F) below 2^64 for every key of the segment).
 * A sub-segment of a feasible segment is feasible (the same line, its
 * intercept moved to the new start, which stays >= first_key 2^F since
 * A >= 0), so growing each segment as far as it goes gives the fewest
 * segments of the class.  Stored: A = floor((lo + hi) / 2) (0 for a one-key
 * segment), C = floor((g + h) / 2) of that A's intercept interval [g, h],
 * anchor = floor(C / 2^F) modulo 2^64 and frac = C mod 2^F.
 */
uint32_t lcref_fit_block_opt(const uint64_t* k, uint32_t nb, uint32_t eps, uint32_t F,
                             uint32_t* seg_start, uint64_t* seg_anchor, uint64_t* seg_A, uint64_t* seg_frac)
{
    if (nb == 0)
        return 0;
    const i128 scale = (i128)1 << F;
    const i128 cap = (i128)1 << (64 - F);
    const i128 first = (i128)k[0];
    const i128 E = (i128)eps;
    uint32_t nseg = 0;
    uint32_t s = 0;
    while (s < nb) {
        /* Lo of key i in the segment starting at s (the start raised), and Up */
#define LO(i) ((i) == s ? ((i128)k[s] - E > first ? (i128)k[s] - E : first) * scale : ((i128)k[i] - E) * scale)
#define UP(i) (((i128)k[i] + E + 1) * scale - 1)
        i128 lo = 0, hi = (i128)1 << 120;
        uint32_t e = s + 1;
        while (e < nb) {
            if ((i128)k[e] - (i128)k[s] + 2 * E + 1 >= cap)
                break;
            i128 nlo = lo, nhi = hi;
            for (uint32_t i = s; i < e; i++) {
                i128 l = ceil_div(LO(e) - UP(i), (i128)(e - i));
                i128 h = floor_div(UP(e) - LO(i), (i128)(e - i));
                if (l > nlo) nlo = l;
                if (h < nhi) nhi = h;
            }
            if (nlo > nhi)
                break;
            lo = nlo;
            hi = nhi;
            e++;
        }
        i128 A = e > s + 1 ? lo + (hi - lo) / 2 : 0;
        i128 g = LO(s), h = UP(s);
        for (uint32_t i = s + 1; i < e; i++) {
            i128 gi = LO(i) - A * (i128)(i - s), hi_ = UP(i) - A * (i128)(i - s);
            if (gi > g) g = gi;
            if (hi_ < h) h = hi_;
        }
#undef LO
#undef UP
        i128 C = g + (h - g) / 2; /* g <= h: A is feasible; C >= first 2^F >= 0 */
        seg_start[nseg] = s;
        seg_anchor[nseg] = (uint64_t)(C >> F);
        seg_A[nseg] = (uint64_t)A;
        seg_frac[nseg] = (uint64_t)(C & (scale - 1));
        nseg++;
        s = e;
    }
    return nseg;
}

static void put_bits(uint8_t* slab, uint64_t bitpos, uint64_t code, int w)
{
    for (int t = 0; t < w; t++) {
        if ((code >> t) & 1u) {
            uint64_t p = bitpos + (uint64_t)t;
            slab[p / 8] |= (uint8_t)(1u << (p % 8));
        }
    }
}

static uint64_t get_bits(const uint8_t* slab, uint64_t bitpos, int w)
{
    uint64_t v = 0;
    for (int t = 0; t < w; t++) {
        uint64_t p = bitpos + (uint64_t)t;
        if ((slab[p / 8] >> (p % 8)) & 1u)
            v |= 1ull << t;
    }
    return v;
}

static void put_le(uint8_t* dst, uint64_t v, int nbytes)
{
    for (int i = 0; i < nbytes; i++)
        dst[i] = (uint8_t)(v >> (8 * i));
}

static uint64_t get_le(const uint8_t* src, int nbytes)
{
    uint64_t v = 0;
    for (int i = 0; i < nbytes; i++)
        v |= (uint64_t)src[i] << (8 * i);
    return v;
}

/* Byte size of the blob that lcref_compress would write, and the segment
 * count, without writing it.  Same steps, no output. */
static int layout_params(uint64_t n, int kb, int log2_block, uint32_t eps, uint32_t F)
{
    if (kb != 4 && kb != 8) return REF_EINVAL;
    if (log2_block < 6 || log2_block > 12) return REF_EINVAL;
    if (eps > 0x7FFFFFFFu) return REF_EINVAL;
    if (F > 32) return REF_EINVAL;
    if (n > (1ull << 48)) return REF_EINVAL;
    return REF_OK;
}

/*
 * Encoder: validate (keys non-decreasing), partition into blocks, fit each
 * block, compute codes, pack, lay out the blob.  out must hold cap bytes;
 * the blob size is returned in *out_bytes (also when cap is too small, with
 * REF_ENOSPC).
 */
int lcref_compress(const void* keys, uint64_t n, int kb, int log2_block, uint32_t eps,
                   uint32_t F, int fit, uint8_t* out, uint64_t cap, uint64_t* out_bytes)
{
    int rc = layout_params(n, kb, log2_block, eps, F);
    if (rc != REF_OK) return rc;
    if (n > 0 && keys == NULL) return REF_EINVAL;
    if (fit < 0 || fit > 2) return REF_EINVAL; /* 0: greedy, 1: fewest anchored, 2: optimal */
    const int fb = fit == 2 ? frac_bytes(F) : 0; /* fraction bytes per segment */

    /* E0: the keys must be sorted (non-decreasing); duplicates are allowed. */
    for (uint64_t i = 1; i < n; i++)
        if (load_key(keys, kb, i) < load_key(keys, kb, i - 1))
            return REF_EUNSORTED;

    const uint64_t B = 1ull << log2_block;
    const uint64_t nblocks = (n + B - 1) / B;
    const int w = lcref_width(eps);
    const uint64_t res_stride = align16((B * (uint64_t)w + 7) / 8);

    /* E1-E3: fit every block; keep the segments. */
    uint32_t* nseg = calloc(nblocks ? nblocks : 1, sizeof(uint32_t));
    uint32_t* starts = malloc((n ? n : 1) * sizeof(uint32_t));
    uint64_t* anchors = malloc((n ? n : 1) * sizeof(uint64_t));
    uint64_t* slopes = malloc((n ? n : 1) * sizeof(uint64_t));
    uint64_t* fracs = calloc(n ? n : 1, sizeof(uint64_t));
    uint64_t* blockkeys = malloc(B * sizeof(uint64_t));
    if (!nseg || !starts || !anchors || !slopes || !fracs || !blockkeys) {
        free(nseg); free(starts); free(anchors); free(slopes); free(fracs); free(blockkeys);
        return REF_ENOSPC;
    }
    uint64_t nseg_total = 0;
    uint32_t max_nseg = 0;
    uint64_t max_area = 0;
    for (uint64_t b = 0; b < nblocks; b++) {
        uint64_t base = b * B;
        uint32_t nb = (uint32_t)((n - base) < B ? (n - base) : B);
        for (uint32_t j = 0; j < nb; j++)
            blockkeys[j] = load_key(keys, kb, base + j);
        /* segments of block b are stored from index base (at most nb of them) */
        if (fit == 2)
            nseg[b] = lcref_fit_block_opt(blockkeys, nb, eps, F, starts + base, anchors + base, slopes + base,
                                          fracs + base);
        else
            nseg[b] = (fit ? lcref_fit_block_min : lcref_fit_block)(blockkeys, nb, eps, F, starts + base,
                                                                    anchors + base, slopes + base);
        nseg_total += nseg[b];
        if (nseg[b] > max_nseg) max_nseg = nseg[b];
    }

    /* Sizes of the per-block segment areas and of the whole blob. */
    const uint64_t off_first = REF_HEADER;
    const uint64_t off_dir = off_first + align16(nblocks * (uint64_t)kb);
    const uint64_t off_res = off_dir + 16 * nblocks;
    const uint64_t off_seg = off_res + nblocks * res_stride;
    uint64_t total = off_seg;
    for (uint64_t b = 0; b < nblocks; b++) {
        uint64_t base = b * B;
        uint64_t first = load_key(keys, kb, base);
        uint64_t maxd = 0, maxa = 0;
        for (uint32_t t = 0; t < nseg[b]; t++) {
            uint64_t dlt = anchors[base + t] - first;
            if (dlt > maxd) maxd = dlt;
            if (slopes[base + t] > maxa) maxa = slopes[base + t];
        }
        uint64_t m = nseg[b];
        uint64_t area = align16(2 * m) + align16((uint64_t)byte_width(maxd) * m) +
                        align16((uint64_t)byte_width(maxa) * m) + align16((uint64_t)fb * m);
        total += area;
        if (area > max_area) max_area = area;
    }
    *out_bytes = total;
    if (cap < total || out == NULL) {
        free(nseg); free(starts); free(anchors); free(slopes); free(fracs); free(blockkeys);
        return REF_ENOSPC;
    }
    memset(out, 0, total);

    /* Header. */
    put_le(out + 0, REF_MAGIC, 4);
    put_le(out + 4, REF_VERSION, 2);
    out[6] = (uint8_t)kb;
    out[7] = (uint8_t)log2_block;
    out[8] = (uint8_t)F;
    out[9] = (uint8_t)w;
    out[10] = fit == 2 ? (uint8_t)REF_FLAG_FRAC : 0;
    put_le(out + 12, eps, 4);
    put_le(out + 16, n, 8);
    put_le(out + 24, nblocks, 8);
    put_le(out + 32, nseg_total, 8);
    put_le(out + 40, max_nseg, 4);
    put_le(out + 44, max_area, 4);
    put_le(out + 48, off_first, 8);
    put_le(out + 56, off_dir, 8);
    put_le(out + 64, off_res, 8);
    put_le(out + 72, res_stride, 8);
    put_le(out + 80, off_seg, 8);
    put_le(out + 88, total, 8);

    /* E4-E6: codes, slabs, directory and segment areas, block by block. */
    uint64_t seg_off = off_seg;
    for (uint64_t b = 0; b < nblocks; b++) {
        uint64_t base = b * B;
        uint32_t nb = (uint32_t)((n - base) < B ? (n - base) : B);
        uint64_t first = load_key(keys, kb, base);
        put_le(out + off_first + b * (uint64_t)kb, first, kb);

        uint32_t m = nseg[b];
        uint64_t maxd = 0, maxa = 0;
        for (uint32_t t = 0; t < m; t++) {
            uint64_t dlt = anchors[base + t] - first;
            if (dlt > maxd) maxd = dlt;
            if (slopes[base + t] > maxa) maxa = slopes[base + t];
        }
        int ab = byte_width(maxd), sb = byte_width(maxa);

        uint8_t* d = out + off_dir + 16 * b;
        put_le(d + 0, seg_off, 8);
        put_le(d + 8, m, 4);
        put_le(d + 12, nb - 1, 2);
        d[14] = (uint8_t)ab;
        d[15] = (uint8_t)sb;

        /* Codes: Delta[i] = K[i] - floor(f(i)) lies in [-eps, eps]; stored +eps. */
        uint8_t* slab = out + off_res + b * res_stride;
        uint32_t t = 0;
        for (uint32_t j = 0; j < nb; j++) {
            while (t + 1 < m && starts[base + t + 1] <= j)
                t++;
            u128 pred = (u128)anchors[base + t] +
                        (((u128)slopes[base + t] * (u128)(j - starts[base + t]) + fracs[base + t]) >> F);
            u128 key = load_key(keys, kb, base + j);
            /* pred - eps <= key <= pred + eps, pred taken modulo 2^64 (an
             * intercept of the optimal fit may pass 2^64): exact modulo 2^64 */
            u128 code = (uint64_t)(key + eps - pred);
            put_bits(slab, (uint64_t)j * (uint64_t)w, (uint64_t)code, w);
        }

        uint8_t* sa = out + seg_off;
        for (uint32_t u = 0; u < m; u++)
            put_le(sa + 2 * (uint64_t)u, starts[base + u], 2);
        sa += align16(2ull * m);
        for (uint32_t u = 0; u < m; u++)
            put_le(sa + (uint64_t)ab * u, anchors[base + u] - first, ab);
        sa += align16((uint64_t)ab * m);
        for (uint32_t u = 0; u < m; u++)
            put_le(sa + (uint64_t)sb * u, slopes[base + u], sb);
        sa += align16((uint64_t)sb * m);
        for (uint32_t u = 0; u < m && fb; u++)
            put_le(sa + (uint64_t)fb * u, fracs[base + u], fb);
        seg_off += align16(2ull * m) + align16((uint64_t)ab * m) + align16((uint64_t)sb * m) +
                   align16((uint64_t)fb * m);
    }

    free(nseg); free(starts); free(anchors); free(slopes); free(fracs); free(blockkeys);
    return REF_OK;
}

/* Header fields, parsed and checked against the layout rules. */
typedef struct {
    uint32_t kb, log2_block, F, w, eps, max_nseg, max_seg_bytes, flags;
    uint64_t n, nblocks, nseg_total, off_first, off_dir, off_res, res_stride, off_seg, bytes;
} ref_header;

static int parse_header(const uint8_t* blob, uint64_t avail, ref_header* h)
{
    if (blob == NULL || avail < REF_HEADER) return REF_EFORMAT;
    if (get_le(blob, 4) != REF_MAGIC || get_le(blob + 4, 2) != REF_VERSION) return REF_EFORMAT;
    h->kb = blob[6];
    h->log2_block = blob[7];
    h->F = blob[8];
    h->w = blob[9];
    h->flags = blob[10];
    if ((h->flags & ~REF_FLAG_FRAC) != 0 || blob[11] != 0) return REF_EFORMAT;
    h->eps = (uint32_t)get_le(blob + 12, 4);
    h->n = get_le(blob + 16, 8);
    h->nblocks = get_le(blob + 24, 8);
    h->nseg_total = get_le(blob + 32, 8);
    h->max_nseg = (uint32_t)get_le(blob + 40, 4);
    h->max_seg_bytes = (uint32_t)get_le(blob + 44, 4);
    h->off_first = get_le(blob + 48, 8);
    h->off_dir = get_le(blob + 56, 8);
    h->off_res = get_le(blob + 64, 8);
    h->res_stride = get_le(blob + 72, 8);
    h->off_seg = get_le(blob + 80, 8);
    h->bytes = get_le(blob + 88, 8);
    if (layout_params(h->n, (int)h->kb, (int)h->log2_block, h->eps, h->F) != REF_OK)
        return REF_EFORMAT;
    if ((int)h->w != lcref_width(h->eps)) return REF_EFORMAT;
    uint64_t B = 1ull << h->log2_block;
    if (h->nblocks != (h->n + B - 1) / B) return REF_EFORMAT;
    if (h->off_first != REF_HEADER) return REF_EFORMAT;
    if (h->off_dir != h->off_first + align16(h->nblocks * h->kb)) return REF_EFORMAT;
    if (h->off_res != h->off_dir + 16 * h->nblocks) return REF_EFORMAT;
    if (h->res_stride != align16((B * h->w + 7) / 8)) return REF_EFORMAT;
    if (h->off_seg != h->off_res + h->nblocks * h->res_stride) return REF_EFORMAT;
    if (h->bytes < h->off_seg || h->bytes > avail) return REF_EFORMAT;
    return REF_OK;
}

/* Independent blob decoder: K[i] = floor(f(i)) + Delta[i] (Sec. II-A), for
 * every i, reading the blob layout described at the top of this file. */
int lcref_decode(const uint8_t* blob, uint64_t avail, void* out, uint64_t out_cap)
{
    ref_header h;
    int rc = parse_header(blob, avail, &h);
    if (rc != REF_OK) return rc;
    if (out_cap < h.n) return REF_ENOSPC;
    const uint64_t B = 1ull << h.log2_block;
    for (uint64_t b = 0; b < h.nblocks; b++) {
        const uint8_t* d = blob + h.off_dir + 16 * b;
        uint64_t seg_off = get_le(d, 8);
        uint32_t m = (uint32_t)get_le(d + 8, 4);
        uint32_t nb = (uint32_t)get_le(d + 12, 2) + 1;
        int ab = d[14], sb = d[15];
        uint64_t expect_nb = (h.n - b * B) < B ? (h.n - b * B) : B;
        if (nb != expect_nb || m == 0 || m > nb) return REF_EFORMAT;
        if (!(ab == 1 || ab == 2 || ab == 4 || ab == 8)) return REF_EFORMAT;
        if (!(sb == 1 || sb == 2 || sb == 4 || sb == 8)) return REF_EFORMAT;
        const int fb = (h.flags & REF_FLAG_FRAC) ? frac_bytes(h.F) : 0;
        uint64_t area = align16(2ull * m) + align16((uint64_t)ab * m) + align16((uint64_t)sb * m) +
                        align16((uint64_t)fb * m);
        if (seg_off < h.off_seg || seg_off + area > h.bytes) return REF_EFORMAT;
        if (m > h.max_nseg || area > h.max_seg_bytes) return REF_EFORMAT;
        const uint8_t* st = blob + seg_off;
        const uint8_t* an = st + align16(2ull * m);
        const uint8_t* sl = an + align16((uint64_t)ab * m);
        const uint8_t* fr = sl + align16((uint64_t)sb * m);
        const uint8_t* slab = blob + h.off_res + b * h.res_stride;
        uint64_t first = get_le(blob + h.off_first + b * h.kb, (int)h.kb);
        for (uint32_t j = 0; j < nb; j++) {
            /* segment of key j: the last one whose start is <= j */
            uint32_t t = 0;
            for (uint32_t u = 0; u < m; u++)
                if (get_le(st + 2ull * u, 2) <= j)
                    t = u;
            uint64_t s = get_le(st + 2ull * t, 2);
            u128 anchor = (u128)first + get_le(an + (uint64_t)ab * t, ab);
            u128 A = get_le(sl + (uint64_t)sb * t, sb);
            u128 frac = fb ? get_le(fr + (uint64_t)fb * t, fb) : 0;
            u128 pred = anchor + ((A * (u128)(j - s) + frac) >> h.F);
            u128 code = get_bits(slab, (uint64_t)j * h.w, (int)h.w);
            u128 key = pred + code - h.eps;
            uint64_t i = b * B + j;
            if (h.kb == 4)
                ((uint32_t*)out)[i] = (uint32_t)key;
            else
                ((uint64_t*)out)[i] = (uint64_t)key;
        }
    }
    return REF_OK;
}

/* Header fields for tests: writes 17 u64 values in the order of ref_header. */
int lcref_header(const uint8_t* blob, uint64_t avail, uint64_t* fields)
{
    ref_header h;
    int rc = parse_header(blob, avail, &h);
    if (rc != REF_OK) return rc;
    uint64_t v[17] = {h.kb, h.log2_block, h.F, h.w, h.eps, h.max_nseg, h.max_seg_bytes, h.n,
                      h.nblocks, h.nseg_total, h.off_first, h.off_dir, h.off_res,
                      h.res_stride, h.off_seg, h.bytes, h.flags};
    memcpy(fields, v, sizeof v);
    return REF_OK;
}
