/*
 * lc.h -- C ABI of the MI355X (gfx950) learned compressor for sorted integer
 * keys (arXiv 2412.10770, "Learned Data Compression: Challenges and
 * Opportunities for the Future").
 *
 * The library encodes a sorted key list K (Def. 1) as an error-bounded
 * piecewise linear model plus bit-packed residuals (Def. 2, Eq. 1, Sec. II-A)
 * and answers queries on the compressed form.  Every entry point works on
 * device memory and only enqueues work on the given stream; nothing here
 * allocates device memory or synchronises (the request server below is the
 * one exception to both, and says so), and the only state kept between
 * calls is a per-device record of kernels whose LDS limit was already
 * raised (guarded by a mutex; the library is reentrant).  The caller owns
 * every buffer.
 *
 * Conventions shared by all entry points:
 *   - keys are unsigned integers of key_bytes = 4 or 8 bytes, little-endian,
 *     in non-decreasing order (duplicates allowed); indices are 0-based;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *   - the return value is 0 (LC_OK) or a negative LC_E* code, detected on the
 *     host before anything is enqueued (nothing is enqueued on error);
 *   - data-dependent problems found on the device are OR-ed into a caller
 *     provided 32-bit flag word (LC_FLAG_*), which the caller zeroes.
 *
 * Blob v1 (the compressed form, little-endian, every region 16-byte aligned,
 * every pad byte zero):
 *   header (128 B): magic "LCB1", version 1, key_bytes, log2_block, frac_bits
 *     F, residual width w, flags (byte 10; bit 0 = LC_BLOB_FLAG_FRAC), eps,
 *     n, nblocks, nseg_total, max_nseg, max_seg_bytes, the byte offsets of
 *     the four regions below, res_stride, blob_bytes;
 *   first_keys[nblocks]   the first key of every block of B = 2^log2_block keys;
 *   dir[nblocks]          16 B each: segment-area offset, segment count,
 *                         key count - 1, anchor and slope byte widths;
 *   residual slabs        block b at off_res + b*res_stride, code j of the
 *                         block in bits [j*w, j*w + w) of an LSB-first stream;
 *   segment areas         per block: u16 start[], anchor - first_key[] and
 *                         slope A[] (1, 2, 4 or 8 bytes each), and with
 *                         LC_BLOB_FLAG_FRAC the intercept fractions frac[]
 *                         (LC_FRAC_BYTES(F) bytes each; none at F = 0).
 * Key i = b*B + j decodes as
 *   anchor[t] + floor((A[t] * (j - start[t]) + frac[t]) / 2^F) + code_j - eps
 * (mod 2^64; frac = 0 without the flag) with t the last segment of block b
 * starting at or before j, i.e. the paper's K[i] = floor(f(i)) + Delta[i]
 * with a fixed-point f.  Without the flag the anchor is the segment's first
 * key; with it, anchor + frac / 2^F is the line's intercept at the start.
 */
#ifndef LC_H
#define LC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lc_status;

#define LC_OK 0
#define LC_EINVAL (-1)   /* null pointer, bad parameter, bad range, n too large */
#define LC_ENOSPC (-2)   /* blob_cap or ws_bytes below what lc_compress_bound gives */
#define LC_EFORMAT (-3)  /* header: bad magic/version or inconsistent fields */
#define LC_EDEVICE (-4)  /* a kernel launch failed (hipGetLastError after launch) */
#define LC_ETOOBIG (-5)  /* lc_compress_noalloc: the workspace would exceed LC_NOALLOC_SCRATCH_BYTES */

#define LC_FLAG_UNSORTED 1u /* compress: keys not non-decreasing; blob is invalid */
#define LC_FLAG_RANGE 2u    /* access: an index >= n; its output slot is 0 */
#define LC_FLAG_INTERNAL 4u /* compress: an internal step limit was hit; blob invalid (a bug) */
#define LC_FLAG_BADLIST 8u  /* batch: a list's keys, blob slot or output lie outside the buffers
                               given, or its eps exceeds the plan's max_eps (the list was skipped),
                               or a block's directory entry is inconsistent with its layout (the
                               block was skipped) */

#define LC_DEFAULT_LOG2_BLOCK 10
#define LC_DEFAULT_FRAC_BITS 0
#define LC_MAX_EPS 0x7FFFFFFFu
#define LC_HEADER_BYTES 128

/* Segment choice of the fit (lc_params.fit).  The first two form anchored
 * segments (anchor = the segment's first key, integer slope A, the midpoint
 * of the segment's feasible slopes):
 *   LC_FIT_GREEDY  each segment grows while some slope keeps all its keys
 *                  within eps (Def. 2, Eq. 1);
 *   LC_FIT_MIN     the fewest segments of that same class per block (the
 *                  optimal-size goal of Sec. II-A within anchored segments):
 *                  among the minimum segmentations, the one whose every
 *                  boundary lies earliest.  Fewer segments, slower fit.
 *   LC_FIT_OPT     the optimal eps-PLA of Sec. II-A in fixed point: lines
 *                  floor((C + A d) / 2^F) with a free integer intercept C
 *                  >= first_key * 2^F and integer A >= 0; each segment grows
 *                  while some (A, C) keeps its keys within eps, which in this
 *                  class gives the fewest segments.  Stored: A = midpoint of
 *                  the feasible slopes, C = midpoint of that A's feasible
 *                  intercepts.  Sets LC_BLOB_FLAG_FRAC; at F = 0 the blob
 *                  carries no fraction array.  One wave per block. */
#define LC_FIT_GREEDY 0
#define LC_FIT_MIN 1
#define LC_FIT_OPT 2

/* Header flag (lc_blob_info.flags): segments carry intercept fractions. */
#define LC_BLOB_FLAG_FRAC 1u
/* Bytes of one intercept fraction for F fractional bits. */
#define LC_FRAC_BYTES(F) ((F) == 0 ? 0u : (F) <= 8 ? 1u : (F) <= 16 ? 2u : 4u)

/* Encoder parameters.
 *   key_bytes  4 or 8
 *   log2_block 6..12 (block size B = 2^log2_block keys; segments never cross
 *              a block)
 *   frac_bits  0..32, fractional bits F of the fixed-point slope A / 2^F
 *              (LC_DEFAULT_FRAC_BITS = 0: integer slopes, the smallest and
 *              fastest blobs measured on every workload here)
 *   fit        LC_FIT_GREEDY (0), LC_FIT_MIN or LC_FIT_OPT
 *   eps        0..LC_MAX_EPS, the error bound of Def. 2; residuals take
 *              w = ceil(log2(2 eps + 1)) bits each (Sec. II-A) */
typedef struct lc_params {
    uint8_t key_bytes;
    uint8_t log2_block;
    uint8_t frac_bits;
    uint8_t fit;
    uint32_t eps;
} lc_params;

/* Host-side copy of a blob's header fields (filled by lc_info). */
typedef struct lc_blob_info {
    uint32_t key_bytes, log2_block, frac_bits, width, eps;
    uint32_t max_nseg;      /* most segments in one block */
    uint32_t max_seg_bytes; /* largest segment area of one block (sizes decode's LDS) */
    uint32_t flags;         /* header byte 10: LC_BLOB_FLAG_FRAC or 0 */
    uint64_t n, nblocks, nseg_total;
    uint64_t off_first, off_dir, off_res, res_stride, off_seg, blob_bytes;
} lc_blob_info;

/* Worst-case sizes for compressing n keys with parameters p (host only,
 * pure).  Sec. II-A: the compressed form K^c = (f, Delta) is the model f
 * (its segments) plus n residuals of w = ceil(log2(2 eps + 1)) bits, so
 * size(K^c) is largest when every block needs the most segments; *blob_max
 * is that size in blob v1.  *ws_bytes: bytes of the device workspace
 * lc_compress needs.  Either output pointer may be NULL.
 * Errors: LC_EINVAL (bad p, p NULL, n > 2^40). */
lc_status lc_compress_bound(uint64_t n, const lc_params* p, uint64_t* blob_max,
                            uint64_t* ws_bytes);

/* Enc of Def. 1: compress n keys at d_keys (device, key_bytes each, sorted)
 * into d_blob (device, blob_cap bytes, 16-byte aligned).  The fit follows
 * Def. 2 / Eq. 1 per block: segments with an integer slope, anchored and
 * chosen greedily or for the fewest segments, or with a free fixed-point
 * intercept (p->fit), residuals bit-packed at
 * ceil(log2(2 eps + 1)) bits (Sec. II-A).
 * d_ws: device workspace of ws_bytes (16-byte aligned), contents scratch.
 * d_blob_bytes: device u64 receiving the blob size (may be NULL).
 * d_flags: device u32 flag word (required); LC_FLAG_UNSORTED is OR-ed in
 * when the keys are not sorted, in which case the blob must not be used.
 * The blob is byte-for-byte deterministic.  Asynchronous on `stream`.
 * Errors: LC_EINVAL, LC_ENOSPC (blob_cap / ws_bytes too small), LC_EDEVICE. */
lc_status lc_compress(const void* d_keys, uint64_t n, const lc_params* p, void* d_blob,
                      uint64_t blob_cap, void* d_ws, uint64_t ws_bytes, uint64_t* d_blob_bytes,
                      uint32_t* d_flags, void* stream);

/* Bytes of the static device scratch of lc_compress_noalloc (per GPU). */
#define LC_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* lc_compress for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops and harnesses that forbid
 * hipMalloc.  Same arguments, results and errors as lc_compress minus the
 * workspace: the library's own static device array of
 * LC_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends) serves as
 * the workspace, and the call allocates nothing.  Limit: the workspace that
 * lc_compress_bound reports for (n, p) must fit in that array, else
 * LC_ETOOBIG and nothing is enqueued (about 3.7e6 keys at 1024-key blocks,
 * 3.0e6 with the optimal fit).  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other host threads)
 * race and must be serialised by the caller; calls in order on one stream
 * are safe.  The first call on a device looks up the array's device
 * address (with that device current); LC_EDEVICE if that fails. */
lc_status lc_compress_noalloc(const void* d_keys, uint64_t n, const lc_params* p, void* d_blob,
                              uint64_t blob_cap, uint64_t* d_blob_bytes, uint32_t* d_flags, void* stream);

/* Parse and check a blob header from host memory (at least 128 bytes, the
 * first bytes of the blob).  The header describes K^c = (f, Delta) of
 * Sec. II-A: the model's segment count and layout, eps and the residual
 * width w, and size(K^c) in bytes (blob_bytes, the numerator of the
 * compression ratio of Def. 1).  Pure host code.
 * Errors: LC_EINVAL (NULL), LC_EFORMAT (magic, version or fields). */
lc_status lc_info(const void* h_header, uint64_t header_bytes, lc_blob_info* out);

/* Dec of Def. 1: write all n keys (key_bytes each) to d_out (device, aligned
 * to key_bytes; 16-byte alignment gives the fastest stores).  d_blob is the
 * device blob described by info; a directory entry inconsistent with the
 * layout makes the decoder skip that block (its keys are not written).
 * Errors: LC_EINVAL (NULL pointer, info inconsistent), LC_EDEVICE. */
lc_status lc_decompress(const void* d_blob, const lc_blob_info* info, void* d_out,
                        void* stream);

/* Dec of Def. 1 restricted to [begin, end): d_out[i - begin] = Dec(K^c)[i]
 * = K[i] (key_bytes each, d_out aligned to key_bytes).  Only the blocks
 * holding the range are read.  0 <= begin <= end <= n, else LC_EINVAL.
 * An empty range enqueues nothing. */
lc_status lc_decompress_range(const void* d_blob, const lc_blob_info* info, uint64_t begin,
                              uint64_t end, void* d_out, void* stream);

/* Random access on the compressed form, the lookup of Sec. II-B: d_out[q]
 * = Dec(K^c)[d_idx[q]] = K[d_idx[q]] (Def. 1) for q < m, each from one
 * block without decoding the others (d_idx: device u64[m]; d_out: device,
 * key_bytes each).  An index >= n writes 0 and ORs LC_FLAG_RANGE into
 * *d_flags (device u32, required).  A directory entry inconsistent with the
 * layout (a corrupt blob) writes 0 and ORs LC_FLAG_BADLIST; no read leaves
 * the blob.  lc_lower_bound, lc_quantile and the server's point requests
 * check the entry the same way (they answer n, 0 and 0 / n for such a block).
 * Errors: LC_EINVAL, LC_EDEVICE. */
lc_status lc_access(const void* d_blob, const lc_blob_info* info, const uint64_t* d_idx,
                    uint64_t m, void* d_out, uint32_t* d_flags, void* stream);

/* lower_bound on the compressed form: d_pos[q] = the smallest i in [0, n]
 * with K[i] >= d_q[q] (n when every key is smaller), for q < m.  d_q holds m
 * keys of key_bytes each; d_pos is device u64[m].  Blocks are located through
 * first_keys and segments through their anchors, the segment-level pruning of
 * Sec. III-A.  Cannot fail on valid input.
 * Errors: LC_EINVAL, LC_EDEVICE. */
lc_status lc_lower_bound(const void* d_blob, const lc_blob_info* info, const void* d_q,
                         uint64_t m, uint64_t* d_pos, void* stream);

/* ---- Queries on the compressed form (Sec. III-A, III-C) --------------------
 */

/* The k-th q-quantile of the list (Sec. III-C: a quantile is one access of
 * the learned encoding), 0-based: d_out[t] = K[min(floor(n * d_k[t] / q),
 * n - 1)] for t < m (d_k: device u64[m]; d_out: key_bytes each).  approx
 * != 0 returns the model's prediction f of that index instead (no residual
 * read; within eps of the key).  n >= 1 and q >= 1, else LC_EINVAL. */
lc_status lc_quantile(const void* d_blob, const lc_blob_info* info, const uint64_t* d_k, uint64_t q, uint64_t m,
                      uint32_t approx, void* d_out, void* stream);

/* Approximate query processing (Sec. III-C): keys [begin, end) decoded from
 * the model alone, without reading the residuals -- d_out[i - begin] =
 * f(i) = anchor + floor(A * (i - start) / 2^F) of i's segment, within eps
 * of K[i] (Def. 2).  Arguments as lc_decompress_range. */
lc_status lc_decompress_approx(const void* d_blob, const lc_blob_info* info, uint64_t begin, uint64_t end,
                               void* d_out, void* stream);

#define LC_SETOP_INTERSECT 1u /* AND: the sorted set of keys in both lists */
#define LC_SETOP_UNION 2u     /* OR: the sorted set of keys in either list */

/* Host, pure: output capacity (keys) and workspace bytes of lc_setop (the
 * list AND / OR of Sec. III-A) for two blobs of the same key width (AND:
 * min(n_a, n_b); OR: n_a + n_b).
 * Errors: LC_EINVAL (bad op, infos inconsistent, key widths differ). */
lc_status lc_setop_bound(const lc_blob_info* a, const lc_blob_info* b, uint32_t op, uint64_t* out_max,
                         uint64_t* ws_bytes);

/* List AND / OR of two compressed lists (Sec. III-A), e.g. posting lists:
 * d_out receives the result keys (sorted, each value once) and *d_count
 * (device u64) their number.  AND decodes the smaller list and probes the
 * larger one in its compressed form: each probe locates one block from the
 * first keys, one segment from the block's anchors and the key inside that
 * segment, so blocks and segments that cannot hold a probe are never read
 * (the segment pruning that replaces skip pointers).  OR decodes both and
 * places every distinct key at its rank.  d_ws: workspace of the size
 * lc_setop_bound gives (16-byte aligned); d_out: out_cap keys, aligned to
 * the key width.  Errors: LC_EINVAL, LC_ENOSPC (out_cap or ws_bytes too
 * small), LC_EDEVICE. */
lc_status lc_setop(uint32_t op, const void* d_blob_a, const lc_blob_info* a, const void* d_blob_b,
                   const lc_blob_info* b, void* d_ws, uint64_t ws_bytes, void* d_out, uint64_t out_cap,
                   uint64_t* d_count, void* stream);

/* ---- Batches of lists ----------------------------------------------------
 * Many sorted lists (e.g. the posting lists of an inverted index, Sec. III-A)
 * compressed or decompressed together: one launch runs the fit over every
 * (list, block) work item, so the cost of a step no longer grows with the
 * number of lists.  Every list gets an ordinary blob v1 in a slot of one
 * buffer: a list's blob is byte-for-byte what lc_compress gives for it.  All
 * lists share key_bytes, log2_block and frac_bits; each has its own eps.
 *
 * The table of lists lives in device memory for the kernels (d_lists) and is
 * prepared on the host by lc_batch_plan.  Every list is checked on the device
 * against the buffers given (key range, blob slot, output range, eps <=
 * max_eps); a list that fails is skipped and LC_FLAG_BADLIST is OR-ed into
 * d_stats[0].
 */

#define LC_BATCH_MAX_CANDIDATES 8

/* One list of a batch (64 bytes). */
typedef struct lc_batch_list {
    uint64_t key_off;   /* index of the list's first key in the concatenated keys (compress)
                           and in the concatenated output (decompress) */
    uint64_t n;         /* keys in the list (may be 0) */
    uint64_t blob_off;  /* byte offset of the list's blob slot in the batch buffer (lc_batch_plan) */
    uint64_t blob_cap;  /* bytes of the slot: the list's lc_compress_bound at max_eps (lc_batch_plan) */
    uint64_t block_off; /* blocks of all earlier lists (lc_batch_plan) */
    uint64_t group_off; /* 4-block groups of all earlier lists (lc_batch_plan) */
    uint32_t eps;       /* the list's error bound, <= max_eps */
    uint32_t reserved[3];
} lc_batch_list;

/* Wave tiling of a batch's greedy fit (lc_batch_params.tiling).  Both give
 * byte-identical blobs; they differ in speed only.
 *   LC_TILING_AUTO   lanes from 16384 blocks in the batch on, rows below
 *   LC_TILING_ROWS   four blocks per wave, 16 lanes evaluating 16 candidate
 *                    keys of one block per step
 *   LC_TILING_LANES  64 blocks per wave, one lane walking each block key by
 *                    key (the residual codes packed by a second pass) */
#define LC_TILING_AUTO 0
#define LC_TILING_ROWS 1
#define LC_TILING_LANES 2

/* Parameters shared by the lists of a batch. */
typedef struct lc_batch_params {
    uint8_t key_bytes, log2_block, frac_bits; /* as lc_params */
    uint8_t tiling;        /* LC_TILING_* (the greedy fit's wave tiling; ignored by the other fits) */
    uint32_t nlists;       /* >= 1 */
    uint32_t max_eps;      /* the largest eps any list may take; sizes the slots */
    uint32_t fit;          /* LC_FIT_* of every list of the batch, as lc_params.fit (0: greedy) */
    uint64_t total_blocks; /* set by lc_batch_plan */
    uint64_t total_groups; /* set by lc_batch_plan */
    uint64_t blob_bytes;   /* set by lc_batch_plan: bytes of the batch buffer */
    uint64_t ws_bytes;     /* set by lc_batch_plan: bytes of the device workspace */
} lc_batch_params;

/* Host, pure: fill blob_off, blob_cap, block_off and group_off of
 * h_lists[0 .. p->nlists) (slots packed in list order, each its list's
 * worst-case size at p->max_eps, the size(K^c) bound of Sec. II-A) and p's
 * totals, for a batch of lists such as the posting lists of Sec. III-A.  key_off, n and eps are
 * left as given.  Errors: LC_EINVAL (bad parameters, NULL). */
lc_status lc_batch_plan(lc_batch_params* p, lc_batch_list* h_lists);

/* Enc of Def. 1 (the fit of Sec. II-A) for every list of a batch, e.g. the
 * posting lists of an inverted index (Sec. III-A).  d_keys: nkeys
 * concatenated keys; d_lists: device
 * copy of the planned table; d_blob: blob_cap bytes (>= p->blob_bytes);
 * d_ws: p->ws_bytes of workspace; d_sizes: device u64[nlists] receiving each
 * list's blob size; d_stats: device u32[2] the caller zeroes: [0] flags
 * (LC_FLAG_*), [1] the largest max_seg_bytes of any list (for
 * lc_batch_decompress).  Three launches: the fit over all work items, a scan
 * per list (directory and header), the segment areas.  Asynchronous.
 * Errors: LC_EINVAL, LC_ENOSPC (blob_cap / ws_bytes), LC_EDEVICE. */
lc_status lc_batch_compress(const void* d_keys, uint64_t nkeys, const lc_batch_list* d_lists,
                            const lc_batch_params* p, void* d_blob, uint64_t blob_cap, void* d_ws,
                            uint64_t ws_bytes, uint64_t* d_sizes, uint32_t* d_stats, void* stream);

/* Size pass of the eps autotuner (the per-partition eps choice of
 * Sec. IV-A, with each list a partition): the exact size(K^c) every list
 * would have at each candidate eps, without writing any blob: d_sizes[c * nlists + l]
 * for candidate h_cands[c] (~0 for a list that does not fit the buffers).
 * h_cands: ncand (1 .. LC_BATCH_MAX_CANDIDATES) strictly increasing values
 * <= p->max_eps.  One fit launch over all (candidate, work item) pairs and
 * one scan launch.  d_sizes: device u64[ncand * nlists]; other buffers as
 * lc_batch_compress (no blob). */
lc_status lc_batch_sizes(const void* d_keys, uint64_t nkeys, const lc_batch_list* d_lists,
                         const lc_batch_params* p, const uint32_t* h_cands, uint32_t ncand, void* d_ws,
                         uint64_t ws_bytes, uint64_t* d_sizes, uint32_t* d_stats, void* stream);

/* Autotuner step (Sec. IV-A: eps set per partition by its space cost): for
 * every list l set d_lists[l].eps to the candidate
 * h_cands[c] with the smallest d_sizes[c * nlists + l] (the sizes of
 * lc_batch_sizes run once per candidate); ties go to the smaller eps.
 * h_cands: ncand (1 .. LC_BATCH_MAX_CANDIDATES) strictly increasing values
 * <= p->max_eps.  One launch, no host synchronisation. */
lc_status lc_batch_pick_eps(lc_batch_list* d_lists, const lc_batch_params* p, const uint64_t* d_sizes,
                            const uint32_t* h_cands, uint32_t ncand, void* stream);

/* Dec of Def. 1 for every list of a batch buffer written by
 * lc_batch_compress with
 * the same table (a list's eps must be the one its blob was written with):
 * list l's keys go to d_out + key_off * key_bytes (nout keys in all; d_out
 * aligned to the key width).  max_seg_bytes: d_stats[1] of that compress; it
 * sizes the on-chip staging of segment areas (any value decodes correctly,
 * smaller ones more slowly).  d_stats: device u32 flag word
 * (LC_FLAG_BADLIST).  Blob contents are trusted as written by the compress.
 * Errors: LC_EINVAL, LC_EDEVICE. */
lc_status lc_batch_decompress(const void* d_blob, uint64_t blob_cap, const lc_batch_list* d_lists,
                              const lc_batch_params* p, uint32_t max_seg_bytes, void* d_out, uint64_t nout,
                              uint32_t* d_stats, void* stream);

/* ---- Request server --------------------------------------------------------
 * A request loop over one device-resident blob with continuous batching:
 * requests are admitted in arrival order while the output arena (the HBM
 * budget for results) has room and a launch slot is free; each launch serves
 * a batch of mixed requests (range decodes, point accesses, lower_bounds) in
 * one kernel; up to max_inflight launches run concurrently on their own
 * streams, and a request that arrives while they run joins the next one.  A
 * request's result is exactly what the single-request entry points give
 * (lc_decompress_range / lc_access / lc_lower_bound), alone or in any mix.
 * The decode of Def. 1 restricted to a range, access (Sec. II-B) and
 * lower_bound (Sec. II-B, III-A) are the operations served.
 */

#define LC_OP_RANGE 1u       /* keys [a, b): (b - a) * key_bytes output bytes */
#define LC_OP_ACCESS 2u      /* K[a]: key_bytes output bytes */
#define LC_OP_LOWER_BOUND 3u /* first i with K[i] >= a (n if none): 8 output bytes (u64) */

/* One request (40 bytes). */
typedef struct lc_request {
    uint32_t op;         /* LC_OP_* */
    uint32_t reserved;
    uint64_t a, b;       /* operands, as listed at LC_OP_* */
    uint64_t arrival_ns; /* scheduled arrival, ns after the start of lc_server_run */
    void* d_dest;        /* optional device pointer: the result is copied there before its
                            arena space is given back; NULL: discarded */
} lc_request;

/* What happened to one request (32 bytes); times in ns after the start. */
typedef struct lc_request_result {
    int64_t admit_ns;    /* admitted: output space reserved, put into a launch */
    int64_t launch_ns;   /* its launch was enqueued */
    int64_t complete_ns; /* its launch (and copy to d_dest) was seen complete */
    int32_t status;      /* LC_OK; LC_EINVAL (bad op / range / index >= n); LC_ENOSPC (result
                            larger than the arena); LC_EDEVICE */
    uint32_t launch;     /* index of the launch that served it */
} lc_request_result;

typedef struct lc_serve_config {
    uint32_t max_batch;    /* requests per launch, 1 .. 65536 */
    uint32_t max_inflight; /* concurrent launches (streams), 1 .. 16 */
} lc_serve_config;

/* Totals of one lc_server_run. */
typedef struct lc_serve_stats {
    uint64_t launches;
    uint64_t max_batch_seen;  /* most requests in one launch */
    uint64_t peak_arena_bytes;
    uint64_t arena_waits;     /* admissions stopped because the arena was full */
} lc_serve_stats;

typedef struct lc_server lc_server; /* opaque */

/* Creates a server (the read path of a compressed key store, Sec. III-B)
 * for the blob at d_blob (parsed header `info`) on the current device.
 * d_arena: arena_bytes (>= 16) of device memory, 16-byte aligned, for
 * request outputs -- the HBM budget.  The blob and the arena
 * stay owned by the caller and must outlive the server.  The server
 * allocates its streams, events, pinned staging and small device request
 * tables here (none later).  Errors: LC_EINVAL, LC_EDEVICE. */
lc_status lc_server_create(const void* d_blob, const lc_blob_info* info, void* d_arena, uint64_t arena_bytes,
                           const lc_serve_config* cfg, lc_server** out);

/* Serves h_reqs[0 .. n) -- range decodes (Def. 1), accesses and
 * lower_bounds (Sec. II-B) on the store of Sec. III-B -- as they arrive (by
 * arrival_ns, measured from the call) and returns when all are complete; h_res[i] describes h_reqs[i].
 * Busy-polls on the calling thread.  stats may be NULL.  Errors: LC_EINVAL
 * (NULL arguments), LC_EDEVICE (a launch failed: in-flight work is drained,
 * unserved requests get status LC_EDEVICE). */
lc_status lc_server_run(lc_server* s, const lc_request* h_reqs, uint64_t n, lc_request_result* h_res,
                        lc_serve_stats* stats);

/* Waits for the server's streams and frees what lc_server_create allocated
 * (the end of the Sec. III-B store's read path). */
lc_status lc_server_destroy(lc_server* s);

/* ---- AND over many pairs of lists of one batch (Sec. III-A) -------------
 * The list AND of lc_setop for every pair of a table, in five launches for
 * all pairs: the probe list of each pair (the shorter one) is decoded into
 * the workspace, every probe key is searched in the other list in its
 * compressed form, and each pair's result (sorted, each key once) is packed
 * at the start of its own output region. */

/* One pair (40 bytes). */
typedef struct lc_list_pair {
    uint32_t a, b;          /* list indices into the batch table */
    uint32_t probe, target; /* set by lc_batch_and_plan: probe = the shorter list */
    uint64_t key_off;       /* set by the plan: output / workspace key offset (probe keys of earlier pairs) */
    uint64_t block_off;     /* set by the plan: probe blocks of earlier pairs */
    uint64_t n;             /* set by the plan: keys of the probe list (capacity of the pair's output) */
} lc_list_pair;

/* Host, pure: plans the many-pair list AND of Sec. III-A.  Fills probe,
 * target, key_off, block_off and n of h_pairs[0 .. npairs) from the host
 * copy of the batch table (as lc_batch_plan left it)
 * and returns the totals and the workspace size of lc_batch_and.  Errors:
 * LC_EINVAL (a list index >= nlists, NULL, bad parameters). */
lc_status lc_batch_and_plan(const lc_batch_params* p, const lc_batch_list* h_lists, lc_list_pair* h_pairs,
                            uint32_t npairs, uint64_t* total_keys, uint64_t* total_blocks, uint64_t* ws_bytes);

/* Runs the plan (list AND of Sec. III-A for every pair): d_pairs is the
 * device copy of the planned table; pair i's
 * result keys go to d_out + key_off (d_out: total_keys keys, aligned to the
 * key width) and their number to d_counts[i] (device u64[npairs]).
 * max_seg_bytes: as lc_batch_decompress.  A pair whose lists do not fit the
 * buffers is skipped with count 0 and LC_FLAG_BADLIST in *d_stats.  Errors:
 * LC_EINVAL, LC_ENOSPC (ws_bytes), LC_EDEVICE. */
lc_status lc_batch_and(const void* d_blob, uint64_t blob_cap, const lc_batch_list* d_lists,
                       const lc_batch_params* p, const lc_list_pair* d_pairs, uint32_t npairs, uint64_t total_keys,
                       uint64_t total_blocks, uint32_t max_seg_bytes, void* d_ws, uint64_t ws_bytes, void* d_out,
                       uint64_t* d_counts, uint32_t* d_stats, void* stream);

/* Static description of a status code. */
const char* lc_strerror(lc_status s);

#ifdef __cplusplus
}
#endif

#endif /* LC_H */
