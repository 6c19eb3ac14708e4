// Internal interface between the C ABI (lc_api.cpp) and the kernels
// (lc_kernels.hip).  Not installed; the public interface is include/lc.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lc.h"

namespace lc {

// Byte layout of one blob v1 plus the encoder parameters, as kernel arguments.
struct Layout {
    uint64_t n, nblocks;
    uint64_t off_first, off_dir, off_res, res_stride, off_seg, blob_bytes;
    uint32_t kb, log2b, F, w, eps, max_nseg, max_seg_bytes;
    uint32_t flags;  // header flags: kFlagFrac for the free-intercept (optimal) fit
    uint32_t fb;     // intercept-fraction bytes per segment (0 without kFlagFrac or at F = 0)
};

// Header flag of blobs whose segments carry a free fixed-point intercept
// (the optimal fit): the anchor delta is floor(C / 2^F) - first key (mod
// 2^64) and a fraction array C mod 2^F follows the slopes.
constexpr uint32_t kFlagFrac = 1;

// Bytes of one intercept fraction (F bits).
inline __host__ __device__ uint32_t frac_bytes(uint32_t F) { return F == 0 ? 0u : F <= 8 ? 1u : F <= 16 ? 2u : 4u; }

// Per-block result of the fit kernel, read by the scan and emit kernels.
struct BlockInfo {
    uint32_t nseg;
    uint32_t seg_bytes;  // bytes of the block's segment area
    uint32_t nkeys;
    uint8_t ab, sb;      // anchor-delta and slope byte widths
    uint16_t pad;
};

// Per-tile (256 blocks) sums and, after the tile scan, the tile's offset.
struct TileSum {
    uint64_t bytes, nseg, off;
    uint32_t max_nseg, max_seg_bytes;
};

// Device workspace of lc_compress, carved from the caller's buffer.
struct Workspace {
    BlockInfo* blk;       // [nblocks]
    TileSum* tiles;       // [ntiles]
    uint16_t* seg_start;  // [nblocks * B]: segment starts, block-major
    uint64_t* seg_delta;  // [nblocks * B]: anchor - first key of the block
    uint64_t* seg_A;      // [nblocks * B]: fixed-point slopes
    uint32_t* seg_frac;   // [nblocks * B]: intercept fractions (optimal fit only, else null)
};

constexpr uint32_t kTileBlocks = 256;
constexpr uint64_t kHeaderBytes = 128;

inline uint64_t align16(uint64_t x) { return (x + 15) & ~uint64_t(15); }
inline uint64_t ntiles_of(uint64_t nblocks) { return (nblocks + kTileBlocks - 1) / kTileBlocks; }

// Parameters of a batch of lists, as kernel arguments.
struct BatchArgs {
    uint32_t kb, log2b, F, nlists, max_eps;
    uint32_t tiling;        // LC_TILING_* of the greedy fit
    uint32_t fit;           // LC_FIT_* of every list
    uint64_t total_blocks, total_groups;
    uint64_t nkeys;         // keys in the concatenated key (compress) / output (decompress) array
    uint64_t blob_cap;      // bytes of the batch buffer
};

// A batch of requests for one launch of the server (device tables).
constexpr uint32_t kServeAccess = 2;       // = LC_OP_ACCESS
constexpr uint32_t kServeLowerBound = 3;   // = LC_OP_LOWER_BOUND
struct ServeRange {                        // decode [a, b) to arena + out_off
    uint64_t a, b, out_off;
    uint64_t item_off;                     // waves of all earlier range requests of the batch
};
struct ServePoint {                        // one access(key) or lower_bound(key) to arena + out_off
    uint64_t key, out_off;
    uint32_t op, pad;
    uint64_t pad2;
};
struct ServeArgs {
    Layout L;
    uint32_t nrange, npoint;
    uint64_t range_items;                  // waves of the range requests (one per block touched)
    uint32_t raw_cap;                      // LDS bytes for a staged segment area (set by launch_serve)
};

// Layout of a parsed blob header, re-checked (lc_api.cpp).
lc_status layout_from_info(const lc_blob_info* info, Layout* L);

// Kernel launchers; each returns the hipError_t of its last launch.
hipError_t launch_compress(const void* d_keys, const Layout& L, uint32_t fit, uint8_t* d_blob, const Workspace& ws,
                           uint64_t* d_blob_bytes, uint32_t* d_flags, hipStream_t stream);
hipError_t launch_decode(const uint8_t* d_blob, const Layout& L, uint64_t begin, uint64_t end,
                         void* d_out, hipStream_t stream, bool approx = false);
// Workspace of a list AND / OR (carved by the host).
struct SetWs {
    void* a_keys;        // decoded keys of A (the probe side for AND)
    void* b_keys;        // decoded keys of B (OR only)
    uint8_t *fa, *fb;    // per-key flags
    uint64_t *PA, *PB;   // OR: exclusive prefix counts, n + 1 entries each
    uint64_t* cnt;       // per-tile counts, then their exclusive scan
    uint64_t* tot;       // two totals
};
constexpr uint64_t kSetTileKeys = 1024;  // keys per tile of the set operations

hipError_t launch_quantile(const uint8_t* d_blob, const Layout& L, const uint64_t* d_k, uint64_t q, uint64_t m,
                           bool approx, void* d_out, hipStream_t stream);
hipError_t launch_setop(uint32_t op, const uint8_t* blob_a, const Layout& La, const uint8_t* blob_b, const Layout& Lb,
                        const SetWs& w, void* out, uint64_t* count, hipStream_t stream);
// Workspace of a batched AND (carved by the host).
struct PairWs {
    void* keys;      // decoded probe keys of every pair
    uint8_t* flags;  // per probe key
    uint64_t* cnt;   // per-tile counts, then their exclusive scan
    uint64_t* tot;   // totals
    uint64_t* P;     // exclusive prefix of the flags, total_keys + 1 entries
};
hipError_t launch_batch_and(const uint8_t* d_blob, const lc_batch_list* d_lists, const BatchArgs& a,
                            const lc_list_pair* d_pairs, uint32_t npairs, uint64_t total_keys, uint64_t total_blocks,
                            uint32_t max_seg_bytes, const PairWs& w, void* d_out, uint64_t* d_counts,
                            uint32_t* d_stats, hipStream_t stream);
hipError_t launch_serve(const uint8_t* d_blob, const ServeArgs& s, const ServeRange* d_ranges, const ServePoint* d_points,
                        uint8_t* d_arena, hipStream_t stream);
hipError_t launch_access(const uint8_t* d_blob, const Layout& L, const uint64_t* d_idx, uint64_t m,
                         void* d_out, uint32_t* d_flags, hipStream_t stream);
hipError_t launch_lower_bound(const uint8_t* d_blob, const Layout& L, const void* d_q, uint64_t m,
                              uint64_t* d_pos, hipStream_t stream);

// Batch fit, scan and emit (sizes_only: the size pass over cands[0 .. ncand)).
hipError_t launch_batch_compress(const void* d_keys, const lc_batch_list* d_lists, const BatchArgs& a,
                                 const uint32_t* cands, uint32_t ncand, uint8_t* d_blob, const Workspace& ws,
                                 uint64_t* d_sizes, uint32_t* d_stats, bool sizes_only, hipStream_t stream);
hipError_t launch_batch_pick(lc_batch_list* d_lists, uint32_t nlists, const uint64_t* d_sizes, const uint32_t* cands,
                             uint32_t ncand, hipStream_t stream);
hipError_t launch_batch_decode(const uint8_t* d_blob, const lc_batch_list* d_lists, const BatchArgs& a,
                               uint32_t max_seg_bytes, void* d_out, uint32_t* d_stats, hipStream_t stream);

}  // namespace lc
