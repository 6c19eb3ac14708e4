// HIP kernels of the learned compressor, written for gfx950 (CDNA4, wave64).
//
// Encode (Def. 1 Enc, Def. 2 / Eq. 1 fit, Sec. II-A residual packing):
//   fit_pack     four key blocks per wave, one per 16-lane DPP row: greedy
//                anchored integer cone, row prefix max/min + ballot over 16
//                candidate keys per step, residual codes OR-ed into an LDS
//                slab, slab stored to the blob
//   tile_reduce  per 256 blocks: segment-area bytes, segment counts
//   tile_scan    one workgroup: exclusive scan over tiles, header, blob size
//   dir_emit     per 256 blocks: in-tile scan -> directory entries
//   fit_lanes    one block per lane, 64 per wave, the same greedy fit walked
//                key by key in lockstep (lists of >= 16384 blocks), then
//   code_pack    one wave per block: residual codes from the segment records
//   fit_min      one wave per block: the fewest segments of the anchored class
//   fit_opt      one wave per block: the optimal fit over free fixed-point
//                intercepts, scanning the two convex hulls per key
//   seg_emit     16 lanes per block: segment SoA in 16-byte chunks
// Decode (Def. 1 Dec, K[i] = floor(f(i)) + Delta[i]):
//   decode_full  staging workgroups stream the blocks' compressed bytes
//                through the on-die cache while the others decode (a full
//                decode or a range, one launch)
//   decode       one wave per block: segment table and residual slab staged
//                in LDS (model arrays read from the blob for large areas),
//                16-byte coalesced stores (the decode part of decode_full;
//                alone for the approximate decode and past the grid limit)
//   touch        the separate staging pass of those cases
//   access       one lane per query, K[i] from the compressed block
//   lower_bound  one lane per query: first_keys -> segment anchors -> the
//                eps window of the model -> search inside it (the segment
//                pruning of Sec. III-A)
// Batches of lists: batch_fit / batch_scan / batch_emit / batch_pick /
//   batch_decode run the same per-block work over all lists of a batch.
// Request server: serve decodes the range blocks and answers the point
//   queries of a batch of requests in one launch.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "lc_launch.h"
#include "lc_search.h"
#include "lc_arith.h"

namespace lc {
namespace {

constexpr uint32_t kMagic = 0x3142434Cu;  // "LCB1"
constexpr uint32_t kVersion = 1;
constexpr uint32_t kFlagUnsorted = 1u;
constexpr uint32_t kFlagRange = 2u;
constexpr uint32_t kFlagBadList = 8u;  // batch: a list outside the buffers, or a corrupt directory entry
constexpr uint64_t kMaxGrid = 1ull << 22;  // workgroups per launch; larger jobs loop

__device__ __forceinline__ uint64_t a16(uint64_t x) { return (x + 15) & ~uint64_t(15); }

__device__ __forceinline__ uint32_t byte_width(uint64_t v)
{
    return v < (1ull << 8) ? 1u : v < (1ull << 16) ? 2u : v < (1ull << 32) ? 4u : 8u;
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

// Element t of a little-endian array of `width`-byte unsigned integers whose
// base is aligned to `width`.
template <typename P8>
__device__ __forceinline__ uint64_t load_w(P8 base, uint32_t t, uint32_t width)
{
    switch (width) {
    case 1: return base[t];
    case 2: return reinterpret_cast<const uint16_t*>(base)[t];
    case 4: return reinterpret_cast<const uint32_t*>(base)[t];
    default: return reinterpret_cast<const uint64_t*>(base)[t];
    }
}

template <int KB>
__device__ __forceinline__ uint64_t load_key(const void* p, uint64_t i)
{
    if constexpr (KB == 4) return reinterpret_cast<const uint32_t*>(p)[i];
    else return reinterpret_cast<const uint64_t*>(p)[i];
}

template <int KB>
__device__ __forceinline__ void store_key(void* p, uint64_t i, uint64_t v)
{
    if constexpr (KB == 4) reinterpret_cast<uint32_t*>(p)[i] = static_cast<uint32_t>(v);
    else reinterpret_cast<uint64_t*>(p)[i] = v;
}

// Inclusive scans across the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_incl_max(uint64_t v)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t t = __shfl_up(v, o, 64);
        if (lane >= (uint32_t)o) v = v > t ? v : t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_incl_min(uint64_t v)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t t = __shfl_up(v, o, 64);
        if (lane >= (uint32_t)o) v = v < t ? v : t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_incl_sum(uint64_t v)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t t = __shfl_up(v, o, 64);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_max(uint64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint64_t t = __shfl_xor(v, o, 64);
        v = v > t ? v : t;
    }
    return v;
}

// Exclusive sum over the threads of a workgroup of NT threads (NT % 64 == 0).
// Returns the exclusive prefix; *total receives the workgroup sum.
template <int NT>
__device__ __forceinline__ uint64_t block_excl_sum(uint64_t v, uint64_t* total)
{
    __shared__ uint64_t s_w[NT / 64];
    const uint32_t lane = lane_id(), wave = threadIdx.x / 64;
    uint64_t incl = wave_incl_sum(v);
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint64_t before = 0, all = 0;
    for (uint32_t k = 0; k < NT / 64; k++) {
        uint64_t x = s_w[k];
        if (k < wave) before += x;
        all += x;
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// Largest power of two <= x (x >= 1).
__device__ __forceinline__ uint32_t pow2_floor(uint32_t x) { return 1u << (31 - __clz(x)); }

// ---------------------------------------------------------------------------
// Encode
// ---------------------------------------------------------------------------

// DPP row shift / broadcast of a 32-bit value (lanes whose source lies
// outside the row read 0; callers only use lanes with a valid source).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t v)
{
    return (uint64_t)dpp32<CTRL>((uint32_t)v) | ((uint64_t)dpp32<CTRL>((uint32_t)(v >> 32)) << 32);
}

// Inclusive max / min scans of u64 across the wave with DPP: row_shr 1, 2,
// 4, 8 inside each row of 16 lanes, then row_bcast 15 and row_bcast 31
// carry row totals into the rows above.
template <bool MAX>
__device__ __forceinline__ uint64_t wave_scan64(uint64_t v)
{
    const uint32_t lane = lane_id(), rl = lane & 15;
    auto op = [](uint64_t a, uint64_t b) { return MAX ? (a > b ? a : b) : (a < b ? a : b); };
    uint64_t u;
    u = dpp64<0x111>(v); if (rl >= 1) v = op(v, u);
    u = dpp64<0x112>(v); if (rl >= 2) v = op(v, u);
    u = dpp64<0x114>(v); if (rl >= 4) v = op(v, u);
    u = dpp64<0x118>(v); if (rl >= 8) v = op(v, u);
    u = dpp64<0x142>(v); if ((lane & 31) >= 16) v = op(v, u);
    u = dpp64<0x143>(v); if (lane >= 32) v = op(v, u);
    return v;
}

// floor(x / d) (and x mod d) for 1 <= d <= 4096 and any u64 x, with
// inv = recip(d) (relative error far below 2^-33): 32-bit halves, each
// quotient estimated in FP64 to within 1 and corrected once from its
// remainder.
// 1 / d to nearly full FP64 precision: the hardware reciprocal is an
// approximation, refined by one Newton-Raphson step (squares its error).
__device__ __forceinline__ double recip_f(double dd)
{
    const double r0 = __builtin_amdgcn_rcp(dd);
    return __builtin_fma(r0, __builtin_fma(-dd, r0, 1.0), r0);
}

__device__ __forceinline__ double recip(uint32_t d) { return recip_f((double)d); }

__device__ __forceinline__ uint64_t div_small(uint64_t x, uint32_t d, double inv, uint32_t* rem = nullptr)
{
    const uint32_t xh = (uint32_t)(x >> 32), xl = (uint32_t)x;
    const double eh = (double)xh * inv;  // clamped: the estimate may pass 2^32 - 1 by a hair
    uint32_t qh = (uint32_t)(eh < 4294967295.0 ? eh : 4294967295.0);
    const int64_t rh0 = (int64_t)xh - (int64_t)qh * d;
    qh = qh - (rh0 < 0) + (rh0 >= (int64_t)d);  // the estimate is within 1 of the quotient
    const int64_t rh = (int64_t)xh - (int64_t)qh * d;
    const uint64_t y = ((uint64_t)rh << 32) | xl;  // < d * 2^32 <= 2^44: exact in FP64
    const double el = (double)y * inv;
    uint32_t ql = (uint32_t)(el < 4294967295.0 ? el : 4294967295.0);
    const int64_t rl0 = (int64_t)y - (int64_t)ql * d;
    const int32_t c = (rl0 >= (int64_t)d) - (rl0 < 0);
    ql += c;
    if (rem) *rem = (uint32_t)(rl0 - (int64_t)c * d);
    return ((uint64_t)qh << 32) | ql;
}

// The block's slope-bound numerators are all below 2^49 when
// (span + eps + 1) 2^F < 2^49, span = last key - first key of the block.
__device__ __forceinline__ bool fast_division_ok(uint64_t span, uint64_t eps, uint32_t F)
{
    const uint64_t lim = F < 49 ? (1ull << (49 - F)) : 0;
    return eps + 1 < lim && span < lim - eps - 1;
}

// max / min of two doubles that are never NaN, without the quieting that
// fmax / fmin add to operands the compiler cannot prove canonical
__device__ __forceinline__ double vmax_f64(double a, double b)
{
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ double vmin_f64(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// c ? a : b per lane as one v_cndmask on the active lanes' mask.  Written
// as asm so that the compiler keeps it a select after the branch that c also
// guards, rather than a move inside that branch (which, for a register a
// pending LDS read writes, would wait for the read).
__device__ __forceinline__ uint32_t sel_u32(uint64_t mask, uint32_t a, uint32_t b)
{
    uint32_t r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(b), "v"(a), "s"(mask));
    return r;
}

__device__ __forceinline__ double sel_f64(uint64_t mask, double a, double b)
{
    const uint32_t lo = sel_u32(mask, (uint32_t)__double_as_longlong(a), (uint32_t)__double_as_longlong(b));
    const uint32_t hi = sel_u32(mask, (uint32_t)(__double_as_longlong(a) >> 32),
                                (uint32_t)(__double_as_longlong(b) >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// v as a double, exactly, for v < 2^52: the mantissa of 2^52 + v holds v.
__device__ __forceinline__ double exact_f64(uint64_t v)
{
    return __longlong_as_double((long long)(0x4330000000000000ull | v)) - 4503599627370496.0;
}

// Slope bounds of one key in exact FP64 integer arithmetic, for blocks whose
// span keeps every numerator below 2^49 (fast_division_ok): Df = D, df = d,
// inv = recip(d) (or 1 for d = 1).  pp = 1 + ceil((D - eps) 2^F / d) when
// D >= eps, else 0 (the P encoding); h = floor(((D + eps + 1) 2^F - 1) / d).
// Each quotient is rounded by one FMA into the mantissa of 2^52, which puts
// it at the floor or one above; its exact FMA remainder corrects it.
__device__ __forceinline__ void bounds_f64(double Df, double epsf, double scf, double df, double inv, double& pp,
                                           double& h)
{
    constexpr double kTwo52 = 4503599627370496.0;
    pp = 0.0;
    if (Df >= epsf) {
        const double x = (Df - epsf) * scf;
        double q = __builtin_fma(x, inv, kTwo52) - kTwo52;
        double r = __builtin_fma(-q, df, x);
        const bool neg = r < 0.0;
        q = neg ? q - 1.0 : q;
        r = neg ? r + df : r;
        pp = q + (r != 0.0 ? 2.0 : 1.0);
    }
    const double y = (Df + epsf + 1.0) * scf - 1.0;
    const double q = __builtin_fma(y, inv, kTwo52) - kTwo52;
    const double r = __builtin_fma(-q, df, y);
    h = r < 0.0 ? q - 1.0 : q;
}

// bounds_f64 that also gives, for D < eps, m = floor((eps - D) 2^F / d) (the
// term of a segment whose lower ends are all negative; mbig otherwise): one
// quotient of |D - eps| 2^F serves both sides, since the lanes of a wave
// that take either side share its instructions anyway.
__device__ __forceinline__ void bounds_m_f64(double Df, double epsf, double scf, double df, double inv,
                                             double mbig, double& pp, double& h, double& m)
{
    constexpr double kTwo52 = 4503599627370496.0;
    const bool up = Df >= epsf;
    const double x = (up ? Df - epsf : epsf - Df) * scf;
    double q = __builtin_fma(x, inv, kTwo52) - kTwo52;
    double r = __builtin_fma(-q, df, x);
    const bool neg = r < 0.0;
    q = neg ? q - 1.0 : q;
    r = neg ? r + df : r;
    pp = up ? q + (r != 0.0 ? 2.0 : 1.0) : 0.0;
    m = up ? mbig : q;
    const double y = (Df + epsf + 1.0) * scf - 1.0;
    const double q2 = __builtin_fma(y, inv, kTwo52) - kTwo52;
    const double r2 = __builtin_fma(-q2, df, y);
    h = r2 < 0.0 ? q2 - 1.0 : q2;
}

// div_fast where the caller has established the 2^49 bound (a uniform flag), else div_small.
__device__ __forceinline__ uint64_t div_pick(bool fast, uint64_t x, uint32_t d, double inv, uint32_t* rem = nullptr)
{
    return fast ? div_fast(x, d, inv, rem) : div_small(x, d, inv, rem);
}

// Inclusive max / min scan of u64 inside each row of 16 lanes (DPP row_shr).
template <bool MAX>
__device__ __forceinline__ uint64_t row_scan64(uint64_t v)
{
    const uint32_t rl = lane_id() & 15;
    auto op = [](uint64_t a, uint64_t b) { return MAX ? (a > b ? a : b) : (a < b ? a : b); };
    uint64_t u;
    u = dpp64<0x111>(v); if (rl >= 1) v = op(v, u);
    u = dpp64<0x112>(v); if (rl >= 2) v = op(v, u);
    u = dpp64<0x114>(v); if (rl >= 4) v = op(v, u);
    u = dpp64<0x118>(v); if (rl >= 8) v = op(v, u);
    return v;
}

// Fit step limit per row: an ordinary step advances the candidate window by
// 16 keys or closes a segment, and a short-segment step closes at least one
// segment or hands the row back to the ordinary step, so 4 * B + 64 steps
// always suffice; hitting the limit would mean an internal error, flagged
// instead of looping on.
constexpr uint32_t kFlagInternal = 4u;
// Candidates per lane of the short-segment step: segments of up to this many
// keys close there (divisions by 1, 2, 4 are shifts, by 3 one division).
constexpr uint32_t kShortWindow = 4;

// Four blocks per wave, one per row of 16 lanes (row r of workgroup w: block
// 4 w + r).  LDS: the four residual slabs (u32[res_stride / 4 + 2] each);
// keys are read from global memory (each block's 1024 keys stay in L1/L2
// while the row works on them).
//
// Greedy anchored cone.  For candidate key e of the segment starting at s
// (d = e - s, D = K[e] - K[s]) the integer slopes A with
// |K[e] - (K[s] + floor(A d / 2^F))| <= eps form
//   [ceil((D - eps) 2^F / d), floor(((D + eps + 1) 2^F - 1) / d)].
// The running intersection is tracked as
//   P = 1 + (largest non-negative lower end), 0 while there is none,
//   H = smallest upper end (never negative: keys are sorted),
// for 16 candidates per step by DPP row scans; the segment ends at the first
// candidate where the intersection is empty or D + eps + 1 reaches
// 2^(64 - F).  Stored slope: floor((lo + hi) / 2) clamped to >= 0.  When a
// segment closes with P = 0 every lower end is negative (all its keys lie
// within eps of the anchor, which happens only for a block's last segment);
// only then is lo = -min_e floor((eps - D) 2^F / d) computed, in one more
// pass over the segment.  Each segment's residual codes (offset by eps) are
// then OR-ed into the row's LDS slab, LSB first, and its record (start,
// anchor - first key, A) goes to the workspace.
// Fits blocks blk0 .. blk0 + 3 of one list (layout L; keys, blob and
// workspace pointers already offset to the list).  SIZES: only the per-block
// segment counts and widths are produced (BlockInfo), nothing else is
// written -- the autotuner's size pass.
template <int KB, bool SIZES>
__device__ __forceinline__ void fit_rows(const void* __restrict__ keys, const Layout& L, uint8_t* __restrict__ blob,
                                         const Workspace& ws, uint32_t* __restrict__ flags, uint64_t blk0)
{
    using KT = typename std::conditional<KB == 4, uint32_t, uint64_t>::type;
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t B = 1u << L.log2b;
    const uint32_t slab_words = (uint32_t)(L.res_stride / 4);
    const uint32_t slab_pitch = slab_words + 4;  // words; keeps every slab 16-byte aligned
    const uint32_t lane = threadIdx.x, row = lane >> 4, r = lane & 15;
    uint32_t* s_slab = reinterpret_cast<uint32_t*>(smem) + row * slab_pitch;

    for (uint32_t i = lane; i < 4 * slab_pitch; i += 64) reinterpret_cast<uint32_t*>(smem)[i] = 0;
    __syncthreads();

    const uint64_t b = blk0 + row;
    const uint64_t base = b << L.log2b;
    const uint32_t nb = b < L.nblocks ? (uint32_t)((L.n - base) < B ? (L.n - base) : B) : 0u;
    const KT* K = reinterpret_cast<const KT*>(keys) + (b < L.nblocks ? base : 0);

    // Keys must be non-decreasing, across the block boundary too.
    bool unsorted = false;
    for (uint32_t j = r; j < nb; j += 16) {
        const KT prev = j ? K[j - 1] : (b ? K[-1] : KT(0));
        unsorted |= K[j] < prev;
    }
    if (__ballot(unsorted) != 0 && lane == 0) atomicOr(flags, kFlagUnsorted);

    const uint64_t eps = L.eps;
    const uint32_t F = L.F, w = L.w;
    const uint64_t wmask = (1ull << w) - 1;  // w <= 32
    const uint64_t lim = F == 0 ? (~0ull - eps) : ((1ull << (64 - F)) - eps - 1);
    const uint64_t first = nb ? (uint64_t)K[0] : 0;
    const uint64_t rec = b << L.log2b;
    const uint32_t row_lane0 = row * 16;
    // one-round divisions when all four blocks of the wave allow them (a wrapped span does not)
    const bool fast = __ballot(!fast_division_ok(nb ? (uint64_t)K[nb - 1] - first : 0, eps, F)) == 0;

    uint32_t s = 0, nseg = 0, e0 = 1;
    uint64_t anchor = first, runP = 0, runH = ~0ull, maxA = 0, maxd = 0;
    bool shortm = false;  // the row's last segment was short: try the short-segment step
    for (uint32_t step = 0; __ballot(s < nb) != 0; step++) {
        if (step >= 4 * B + 64) {
            if (lane == 0) atomicOr(flags, kFlagInternal);
            break;
        }
        const bool open = s < nb;
        if (__ballot(open && !shortm) == 0) {
            // Short-segment step (every open row of the wave asked for it):
            // lane r takes key a = s + r as a possible anchor and evaluates
            // candidates a + 1 .. a + kShortWindow, which gives the greedy
            // length of a segment starting at a (1 .. kShortWindow keys, or 0
            // for more).  Walking the chain s -> s + len -> ... closes up to
            // 16 segments at once; a long one hands the row back to the
            // ordinary step.  Bounds as in the ordinary step; divisions by a
            // power of two are shifts.
            const uint32_t a = s + r;
            const bool has = open && a < nb;
            const uint64_t Ka = has ? (uint64_t)K[a] : 0;
            constexpr uint32_t W = kShortWindow;
            uint64_t Pc[W], Hc[W], Dc[W];
            bool okc[W];
#pragma unroll
            for (uint32_t k = 0; k < W; k++) {
                const uint32_t d = k + 1;
                Pc[k] = 0;
                Hc[k] = ~0ull;
                Dc[k] = 0;
                okc[k] = has && a + d < nb;
                if (okc[k]) {
                    const uint64_t D = (uint64_t)K[a + d] - Ka;
                    Dc[k] = D;
                    okc[k] = D < lim;
                    if (okc[k]) {
                        const uint64_t x = (D - eps) << F, y = ((D + eps + 1) << F) - 1;
                        if ((d & (d - 1)) == 0) {
                            const uint32_t sh = 31 - __clz(d);
                            if (D >= eps) Pc[k] = (x >> sh) + ((x & (d - 1)) != 0) + 1;
                            Hc[k] = y >> sh;
                        } else {
                            const double inv = recip(d);
                            if (D >= eps) {
                                uint32_t rem;
                                const uint64_t q = div_pick(fast, x, d, inv, &rem);
                                Pc[k] = q + (rem != 0) + 1;
                            }
                            Hc[k] = div_pick(fast, y, d, inv);
                        }
                    }
                }
            }
            // prefix intersections; len = keys of the greedy segment at a (0: more than W)
            uint64_t Qp = Pc[0], Gp = Hc[0];
            uint32_t len = okc[0] ? 0u : 1u;
            uint64_t Pf = 0, Hf = ~0ull;
            if (okc[0]) { Pf = Pc[0]; Hf = Hc[0]; }
#pragma unroll
            for (uint32_t k = 1; k < W; k++) {
                const uint64_t Qn = Qp > Pc[k] ? Qp : Pc[k], Gn = Gp < Hc[k] ? Gp : Hc[k];
                const bool join = okc[k] && (Qn == 0 || Qn - 1 <= Gn);
                if (len == 0 && !join) {
                    len = k + 1;  // candidates 1 .. k joined
                } else if (len == 0) {
                    Pf = Qn;
                    Hf = Gn;
                }
                Qp = Qn;
                Gp = Gn;
            }
            // walk the chain from anchor s (row-uniform cur)
            uint32_t cur = 0, path = 0;
            bool walking = open, hit_long = false;
            for (uint32_t it = 0; it < 16; it++) {
                const bool live = walking && cur < 16 && s + cur < nb;
                if (__ballot(live) == 0) break;
                const uint32_t lc = __shfl(len, row_lane0 + (cur & 15), 64);
                if (live) {
                    if (lc == 0) {
                        walking = false;
                        hit_long = true;
                    } else {
                        path |= 1u << cur;
                        cur += lc;
                    }
                } else {
                    walking = false;
                }
            }
            const bool mine = open && ((path >> r) & 1u);
            uint64_t A = 0;
            if (mine && len >= 2) {
                if (Pf != 0) {
                    const uint64_t lo = Pf - 1;
                    A = lo + (Hf - lo) / 2;
                } else {
                    // all lower ends negative: lo = -M, M = min floor((eps - D) 2^F / d)
                    uint64_t M = ~0ull;
#pragma unroll
                    for (uint32_t k = 0; k + 1 < W; k++) {
                        if (k + 1 < len) {
                            const uint32_t d = k + 1;
                            const uint64_t z = (eps - Dc[k]) << F;
                            const uint64_t m = (d & (d - 1)) == 0 ? z >> (31 - __clz(d)) : div_pick(fast, z, d, recip(d));
                            M = m < M ? m : M;
                        }
                    }
                    A = Hf >= M ? (Hf - M) / 2 : 0;
                }
            }
            if (mine) {
                const uint32_t idx = nseg + __popc(path & ((1u << r) - 1u));
                if (!SIZES) {
                    ws.seg_start[rec + idx] = (uint16_t)a;
                    ws.seg_delta[rec + idx] = Ka - first;
                    ws.seg_A[rec + idx] = A;
                    if (w != 0) {
                        for (uint32_t k = 0; k < len; k++) {
                            const uint32_t j = a + k;
                            const uint64_t pred = Ka + ((A * (uint64_t)k) >> F);
                            const uint64_t code = ((uint64_t)K[j] - pred + eps) & wmask;
                            const uint32_t bitpos = j * w;
                            const uint32_t wd = bitpos >> 5, sh = bitpos & 31;
                            const uint64_t v = code << sh;
                            atomicOr(&s_slab[wd], (uint32_t)v);
                            if (sh + w > 32) atomicOr(&s_slab[wd + 1], (uint32_t)(v >> 32));
                        }
                    }
                }
            }
            // row maxima of the closed segments' slopes and anchor deltas
            uint64_t mA = mine ? A : 0, mD = mine ? Ka - first : 0;
            mA = row_scan64<true>(mA);
            mD = row_scan64<true>(mD);
            mA = __shfl(mA, row_lane0 + 15, 64);
            mD = __shfl(mD, row_lane0 + 15, 64);
            if (open) {
                maxA = mA > maxA ? mA : maxA;
                maxd = mD > maxd ? mD : maxd;
                nseg += __popc(path);
                s += cur;
                e0 = s + 1;
                runP = 0;
                runH = ~0ull;
                if (s < nb) anchor = K[s];
                if (hit_long) shortm = false;
            }
            continue;
        }
        const uint32_t e = e0 + r;
        const bool valid = open && e < nb;
        uint64_t P = 0, H = ~0ull;
        bool capped = false;
        if (valid) {
            const uint32_t d = e - s;
            const uint64_t D = (uint64_t)K[e] - anchor;
            capped = D >= lim;
            if (!capped) {
                const double inv = recip(d);
                if (D >= eps) {
                    uint32_t rem;
                    const uint64_t q = div_pick(fast, (D - eps) << F, d, inv, &rem);
                    P = q + (rem != 0) + 1;  // 1 + ceil((D - eps) 2^F / d)
                }
                H = div_pick(fast, ((D + eps + 1) << F) - 1, d, inv);
            }
        }
        P = row_scan64<true>(P);
        H = row_scan64<false>(H);
        P = P > runP ? P : runP;
        H = H < runH ? H : runH;
        const bool fail = valid && (capped || (P != 0 && P - 1 > H));
        const uint32_t fm = (uint32_t)(__ballot(fail) >> row_lane0) & 0xFFFFu;
        // f: candidates of this step that join the segment
        const uint32_t avail = e0 < nb ? (nb - e0 < 16 ? nb - e0 : 16u) : 0u;
        const uint32_t f = fm ? (uint32_t)__builtin_ctz(fm) : avail;
        const uint32_t src = row_lane0 + (f ? f - 1 : 0);
        const uint64_t Pl = __shfl(P, src, 64), Hl = __shfl(H, src, 64);
        const uint64_t Pf = f ? Pl : runP, Hf = f ? Hl : runH;
        const bool closes = open && (fm != 0 || e0 + 16 >= nb);
        if (open && !closes) {
            runP = Pf;
            runH = Hf;
            e0 += 16;
        }
        if (closes) {
            const uint32_t e_end = e0 + f;
            uint64_t A = 0;
            if (e_end > s + 1) {
                if (Pf != 0) {
                    const uint64_t lo = Pf - 1;
                    A = lo + (Hf - lo) / 2;
                } else {
                    // all lower ends negative: lo = -M, M = min floor((eps - D) 2^F / d)
                    uint64_t M = ~0ull;
                    for (uint32_t j = s + 1 + r; j < e_end; j += 16) {
                        const uint32_t d = j - s;
                        const uint64_t D = (uint64_t)K[j] - anchor;
                        const uint64_t m = div_pick(fast, (eps - D) << F, d, recip(d));
                        M = m < M ? m : M;
                    }
                    for (int o = 8; o > 0; o >>= 1) {
                        const uint64_t t = __shfl_xor(M, o, 16);
                        M = t < M ? t : M;
                    }
                    A = Hf >= M ? (Hf - M) / 2 : 0;  // floor((-M + H) / 2), clamped
                }
            }
            if (!SIZES && r == 0) {
                ws.seg_start[rec + nseg] = (uint16_t)s;
                ws.seg_delta[rec + nseg] = anchor - first;
                ws.seg_A[rec + nseg] = A;
            }
            if (!SIZES && w != 0) {
                for (uint32_t j = s + r; j < e_end; j += 16) {
                    const uint64_t pred = anchor + ((A * (uint64_t)(j - s)) >> F);
                    const uint64_t code = ((uint64_t)K[j] - pred + eps) & wmask;
                    const uint32_t bitpos = j * w;
                    const uint32_t wd = bitpos >> 5, sh = bitpos & 31;
                    const uint64_t v = code << sh;
                    atomicOr(&s_slab[wd], (uint32_t)v);
                    if (sh + w > 32) atomicOr(&s_slab[wd + 1], (uint32_t)(v >> 32));
                }
            }
            maxA = A > maxA ? A : maxA;
            maxd = anchor - first;
            nseg++;
            shortm = e_end - s <= kShortWindow;
            s = e_end;
            e0 = s + 1;
            runP = 0;
            runH = ~0ull;
            if (s < nb) anchor = K[s];
        }
    }
    __syncthreads();

    if (nb) {
        if (!SIZES) {
            uint4* dst = reinterpret_cast<uint4*>(blob + L.off_res + b * L.res_stride);
            const uint4* src4 = reinterpret_cast<const uint4*>(s_slab);
            for (uint32_t c = r; c < slab_words / 4; c += 16) dst[c] = src4[c];
        }
        if (r == 0) {
            if (!SIZES) store_key<KB>(blob + L.off_first, b, first);
            const uint32_t ab = byte_width(maxd), sb = byte_width(maxA);  // anchors grow with t
            BlockInfo bi;
            bi.nseg = nseg;
            bi.seg_bytes = (uint32_t)(a16(2ull * nseg) + a16((uint64_t)ab * nseg) + a16((uint64_t)sb * nseg));
            bi.nkeys = nb;
            bi.ab = (uint8_t)ab;
            bi.sb = (uint8_t)sb;
            bi.pad = 0;
            ws.blk[b] = bi;
        }
    }
}

template <int KB>
__global__ __launch_bounds__(64) void fit_pack_kernel(const void* __restrict__ keys, Layout L,
                                                       uint8_t* __restrict__ blob, Workspace ws,
                                                       uint32_t* __restrict__ flags, uint64_t blk0)
{
    fit_rows<KB, false>(keys, L, blob, ws, flags, blk0 + (uint64_t)blockIdx.x * 4);
}

// ---------------------------------------------------------------------------
// Fewest-segment fit within the anchored class, one block per wave (a
// workgroup of 64 lanes).  Same segments, slopes and codes as the greedy fit
// would store for the chosen boundaries; only the boundaries differ, so the
// blob format and every decoder are unchanged.
//
// reach[s] is where the greedy segment anchored at s ends: [s, e) is a
// feasible segment exactly when e <= reach[s].  Going backwards from the end
// of the block, each boundary is the smallest s whose reach covers the
// boundary after it; that chain has the fewest segments, and among minimum
// segmentations every one of its boundaries lies earliest.  With
// PM(s) = max(reach[0..s]) non-decreasing, "smallest s with reach[s] >= b"
// is "smallest s with PM(s) >= b", a search in a sorted array.
//
// Phase 1a: anchor 0's reach by the whole wave, 64 candidates per step (DPP
// scans of the slope bounds, as the greedy fit's ordinary step); a block
// that one segment covers is done.  Phase 1b: lane t walks the cones of
// anchors t, t + 64, ... one candidate per step; an anchor whose reach is
// the end of the block covers every boundary, so anchors past the first such
// one are skipped.  Phase 2: PM in place, then the chain: per boundary, one
// 64-way pass over chunk ends and one inside the chunk found.  Phase 3: each
// segment's slope interval, midpoint slope (as in the greedy fit), record and
// residual codes; segments of up to kMinSerialLen keys one per lane, longer
// ones by the whole wave.
// When (span of the block + eps + 1) 2^F < 2^49 every numerator of the
// block's slope bounds fits a one-round FP64 division (block-uniform branch).
// LDS: misc u32[4] | keys KT[B] | slab u32[res_stride / 4 + 4] | PM u16[B] |
// boundaries u16[B + 1].
constexpr uint32_t kMinLanes = 64;
constexpr uint32_t kMinSerialLen = 48;

__device__ __forceinline__ uint64_t wave_max64(uint64_t v) { return __shfl(wave_scan64<true>(v), 63, 64); }
__device__ __forceinline__ uint64_t wave_min64(uint64_t v) { return __shfl(wave_scan64<false>(v), 63, 64); }

struct ConeArgs {
    uint64_t eps;
    uint32_t F;
    bool fast;  // every numerator below 2^49
};

__device__ __forceinline__ uint64_t div_cone(const ConeArgs& c, uint64_t x, uint32_t d, double inv,
                                             uint32_t* rem = nullptr)
{
    return div_pick(c.fast, x, d, inv, rem);
}

// Slope bounds of key e for the segment anchored at s (D = K[e] - K[s] below
// the cap, d = e - s): P = 1 + ceil((D - eps) 2^F / d) if D >= eps, else 0;
// H = floor(((D + eps + 1) 2^F - 1) / d).
__device__ __forceinline__ void cone_bounds(const ConeArgs& c, uint64_t D, uint32_t d, uint64_t& P, uint64_t& H)
{
    const double inv = recip(d);
    P = 0;
    if (D >= c.eps) {
        uint32_t rem;
        const uint64_t q = div_cone(c, (D - c.eps) << c.F, d, inv, &rem);
        P = q + (rem != 0) + 1;
    }
    H = div_cone(c, ((D + c.eps + 1) << c.F) - 1, d, inv);
}

// Stored slope from the interval (P, H) of a segment of two or more keys;
// when every lower end is negative (P = 0), lo = -M with M the minimum of
// floor((eps - D) 2^F / d) over the segment's keys.
__device__ __forceinline__ uint64_t mid_slope(uint64_t P, uint64_t H, uint64_t M)
{
    if (P != 0) {
        const uint64_t lo = P - 1;
        return lo + (H - lo) / 2;
    }
    return H >= M ? (H - M) / 2 : 0;  // floor((H - M) / 2), clamped at 0
}

// Block b of a list (keys, L, blob slot, workspace of the list); SIZES: the
// size pass, block info only (no records, slab or first key written).
template <int KB, bool SIZES>
__device__ __forceinline__ void fit_min_block(const void* __restrict__ keys, const Layout L,
                                              uint8_t* __restrict__ blob, const Workspace& ws,
                                              uint32_t* __restrict__ flags, uint64_t b)
{
    using KT = typename std::conditional<KB == 4, uint32_t, uint64_t>::type;
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t B = 1u << L.log2b;
    const uint32_t lane = threadIdx.x;
    const uint64_t base = b << L.log2b;
    const uint32_t nb = (L.n - base) < B ? (uint32_t)(L.n - base) : B;  // >= 1
    const KT* Kg = reinterpret_cast<const KT*>(keys) + base;

    uint32_t* s_full = reinterpret_cast<uint32_t*>(smem);  // first anchor known to reach nb
    KT* sk = reinterpret_cast<KT*>(smem + 16);
    uint32_t* s_slab = reinterpret_cast<uint32_t*>(smem + 16 + KB * B);
    const uint32_t slab_words = (uint32_t)(L.res_stride / 4);
    uint16_t* pm = reinterpret_cast<uint16_t*>(smem + 16 + KB * B + L.res_stride + 16);
    uint16_t* bnd = pm + ((2 * B + 15) & ~15u) / 2;

    bool unsorted = false;
    for (uint32_t j = lane; j < nb; j += kMinLanes) {
        const KT k = Kg[j];
        const KT prev = j ? Kg[j - 1] : (b ? Kg[-1] : KT(0));
        unsorted |= k < prev;
        sk[j] = k;
        pm[j] = 0;
    }
    for (uint32_t i = lane; i < slab_words + 4; i += kMinLanes) s_slab[i] = 0;
    if (lane == 0) *s_full = nb;
    if (__ballot(unsorted) != 0 && lane == 0) atomicOr(flags, kFlagUnsorted);
    __syncthreads();

    const uint64_t eps = L.eps;
    const uint32_t F = L.F, w = L.w;
    const uint64_t wmask = (1ull << w) - 1;
    const uint64_t lim = F == 0 ? (~0ull - eps) : ((1ull << (64 - F)) - eps - 1);
    const uint64_t first = (uint64_t)sk[0];
    ConeArgs ca;
    ca.eps = eps;
    ca.F = F;
    ca.fast = fast_division_ok((uint64_t)sk[nb - 1] - first, eps, F);  // a wrapped span takes div_small

    // Phase 1a: anchor 0 by the whole wave.
    uint32_t r0 = nb;
    {
        uint64_t runP = 0, runH = ~0ull;
        for (uint32_t e0 = 1; e0 < nb; e0 += kMinLanes) {
            const uint32_t e = e0 + lane;
            const bool valid = e < nb;
            uint64_t P = 0, H = ~0ull;
            bool capped = false;
            if (valid) {
                const uint64_t D = (uint64_t)sk[e] - first;
                capped = D >= lim;
                if (!capped) cone_bounds(ca, D, e, P, H);
            }
            P = wave_scan64<true>(P);
            H = wave_scan64<false>(H);
            P = P > runP ? P : runP;
            H = H < runH ? H : runH;
            const uint64_t fm = __ballot(valid && (capped || (P != 0 && P - 1 > H)));
            if (fm != 0) {
                r0 = e0 + (uint32_t)__builtin_ctzll(fm);
                break;
            }
            runP = __shfl(P, 63, 64);
            runH = __shfl(H, 63, 64);
        }
    }
    if (lane == 0) {
        pm[0] = (uint16_t)r0;
        if (r0 == nb) *s_full = 0;
    }
    __syncthreads();

    // Phase 1b: the other anchors, one walk per lane, up to the first that reaches nb.
    if (r0 < nb) {
        const uint32_t per_lane = (nb + kMinLanes - 1) / kMinLanes;
        const uint32_t step_cap = per_lane * (nb + 1) + 64;
        uint32_t s = lane ? lane : kMinLanes, e = s + 1, steps = 0;
        uint64_t Ka = s < nb ? (uint64_t)sk[s] : 0, P = 0, H = ~0ull;
        constexpr double kBig = 1.8e19;  // no upper end yet: above every real bound (< 2^49)
        const double epsf = (double)eps, scf = (double)(1ull << F);
        double Pf = 0.0, Hf = kBig, inv = 1.0;  // the exact FP64 walk (ca.fast); inv = recip(e - s)
        while (s < nb) {
            if (++steps > step_cap) {
                atomicOr(flags, kFlagInternal);
                break;
            }
            bool stop = e >= nb;
            if (!stop) {
                if (ca.fast) {  // block-uniform; no cap in such blocks
                    const double inv_next = recip(e - s + 1);
                    double pp, h;
                    bounds_f64(exact_f64((uint64_t)sk[e] - Ka), epsf, scf, (double)(e - s), inv, pp, h);
                    const double Pn = pp > Pf ? pp : Pf, Hn = h < Hf ? h : Hf;
                    stop = Pn != 0.0 && Pn - 1.0 > Hn;
                    if (!stop) {
                        Pf = Pn;
                        Hf = Hn;
                        inv = inv_next;
                        e++;
                    }
                } else {
                    const uint64_t D = (uint64_t)sk[e] - Ka;
                    stop = D >= lim;
                    if (!stop) {
                        uint64_t p, h;
                        cone_bounds(ca, D, e - s, p, h);
                        const uint64_t Pn = p > P ? p : P, Hn = h < H ? h : H;
                        stop = Pn != 0 && Pn - 1 > Hn;
                        if (!stop) {
                            P = Pn;
                            H = Hn;
                            e++;
                        }
                    }
                }
            }
            if (stop) {
                pm[s] = (uint16_t)e;
                if (e == nb) atomicMin(s_full, s);
                s += kMinLanes;
                if (s >= nb || s > __hip_atomic_load(s_full, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                    break;
                Ka = sk[s];
                e = s + 1;
                P = 0;
                H = ~0ull;
                Pf = 0.0;
                Hf = kBig;
                inv = 1.0;
            }
        }
    }
    __syncthreads();

    // Phase 2a: PM = running max of reach, in place; lane t owns entries
    // [t c, t c + c).  Values are at most nb <= 4096.
    {
        const uint32_t c = (nb + kMinLanes - 1) / kMinLanes;
        const uint32_t j0 = lane * c < nb ? lane * c : nb, j1 = j0 + c < nb ? j0 + c : nb;
        uint32_t run = 0;
        for (uint32_t j = j0; j < j1; j++) run = pm[j] > run ? pm[j] : run;
        const uint32_t incl = (uint32_t)wave_scan64<true>(run);
        uint32_t acc = (uint32_t)__shfl_up((int)incl, 1, 64);
        if (lane == 0) acc = 0;
        for (uint32_t j = j0; j < j1; j++) {
            acc = pm[j] > acc ? pm[j] : acc;
            pm[j] = (uint16_t)acc;
        }
    }
    __syncthreads();

    // Phase 2b: the chain of boundaries, nb = bnd[0] > bnd[1] > ... > bnd[m] = 0.
    uint32_t m = 0;
    {
        const uint32_t stride = (nb + 63) / 64;
        uint32_t cur = nb;
        if (lane == 0) bnd[0] = (uint16_t)nb;
        while (cur > 0 && m < nb) {
            const uint32_t p1 = (lane + 1) * stride - 1 < nb ? (lane + 1) * stride - 1 : nb - 1;
            const uint64_t b1 = __ballot(pm[p1] >= cur);
            if (b1 == 0) break;  // cannot happen: pm[nb - 1] = nb
            const uint32_t f = (uint32_t)__builtin_ctzll(b1);  // the chunk holding the answer
            const uint32_t p2 = f * stride + lane;
            const uint64_t b2 = __ballot(lane < stride && p2 < nb && pm[p2] >= cur);
            if (b2 == 0) break;  // cannot happen: the chunk's last entry qualifies
            const uint32_t nxt = f * stride + (uint32_t)__builtin_ctzll(b2);
            if (nxt >= cur) break;  // cannot happen: PM(cur - 1) >= cur
            cur = nxt;
            m++;
            if (lane == 0) bnd[m] = (uint16_t)cur;
        }
        if (cur != 0) {
            m = 0;  // no blob: flagged
            if (lane == 0) atomicOr(flags, kFlagInternal);
        }
    }
    __syncthreads();

    // Phase 3: slopes, records and codes of the m segments (segment t is
    // [bnd[m - t], bnd[m - t - 1])).
    const uint64_t rec = b << L.log2b;
    uint64_t maxA = 0;
    auto emit = [&](uint32_t t, uint32_t s, uint64_t anchor, uint64_t A) {
        if (SIZES) return;
        ws.seg_start[rec + t] = (uint16_t)s;
        ws.seg_delta[rec + t] = anchor - first;
        ws.seg_A[rec + t] = A;
    };
    auto put_code = [&](uint32_t j, uint32_t s, uint64_t anchor, uint64_t A) {
        if (SIZES) return;
        const uint64_t pred = anchor + ((A * (uint64_t)(j - s)) >> F);
        const uint64_t code = ((uint64_t)sk[j] - pred + eps) & wmask;
        const uint32_t bitpos = j * w;
        const uint32_t wd = bitpos >> 5, sh = bitpos & 31;
        const uint64_t v = code << sh;
        atomicOr(&s_slab[wd], (uint32_t)v);
        if (sh + w > 32) atomicOr(&s_slab[wd + 1], (uint32_t)(v >> 32));
    };
    for (uint32_t t0 = 0; t0 < m; t0 += kMinLanes) {
        const uint32_t t = t0 + lane;
        bool is_long = false;
        if (t < m) {
            const uint32_t s = bnd[m - t], e = bnd[m - t - 1];
            is_long = e - s > kMinSerialLen;
            if (!is_long) {
                const uint64_t anchor = sk[s];
                uint64_t P = 0, H = ~0ull, A = 0;
                for (uint32_t j = s + 1; j < e; j++) {
                    uint64_t p, h;
                    cone_bounds(ca, (uint64_t)sk[j] - anchor, j - s, p, h);
                    P = p > P ? p : P;
                    H = h < H ? h : H;
                }
                if (e > s + 1) {
                    uint64_t M = ~0ull;
                    if (P == 0)
                        for (uint32_t j = s + 1; j < e; j++) {
                            const uint32_t d = j - s;
                            const uint64_t mm = div_cone(ca, (eps - ((uint64_t)sk[j] - anchor)) << F, d, recip(d));
                            M = mm < M ? mm : M;
                        }
                    A = mid_slope(P, H, M);
                }
                emit(t, s, anchor, A);
                maxA = A > maxA ? A : maxA;
                if (w != 0)
                    for (uint32_t j = s; j < e; j++) put_code(j, s, anchor, A);
            }
        }
        for (uint64_t lm = __ballot(is_long); lm != 0; lm &= lm - 1) {
            const uint32_t tl = t0 + (uint32_t)__builtin_ctzll(lm);
            const uint32_t s = bnd[m - tl], e = bnd[m - tl - 1];
            const uint64_t anchor = sk[s];
            uint64_t P = 0, H = ~0ull;
            for (uint32_t j = s + 1 + lane; j - lane < e; j += kMinLanes) {
                if (j < e) {
                    uint64_t p, h;
                    cone_bounds(ca, (uint64_t)sk[j] - anchor, j - s, p, h);
                    P = p > P ? p : P;
                    H = h < H ? h : H;
                }
            }
            P = wave_max64(P);
            H = wave_min64(H);
            uint64_t M = ~0ull;
            if (P == 0) {
                for (uint32_t j = s + 1 + lane; j < e; j += kMinLanes) {
                    const uint32_t d = j - s;
                    const uint64_t mm = div_cone(ca, (eps - ((uint64_t)sk[j] - anchor)) << F, d, recip(d));
                    M = mm < M ? mm : M;
                }
                M = wave_min64(M);
            }
            const uint64_t A = mid_slope(P, H, M);
            if (lane == 0) emit(tl, s, anchor, A);
            maxA = A > maxA ? A : maxA;
            if (w != 0)
                for (uint32_t j = s + lane; j < e; j += kMinLanes) put_code(j, s, anchor, A);
        }
    }
    maxA = wave_max64(maxA);
    __syncthreads();

    if (!SIZES) {
        uint4* dst = reinterpret_cast<uint4*>(blob + L.off_res + b * L.res_stride);
        const uint4* src4 = reinterpret_cast<const uint4*>(s_slab);
        for (uint32_t c = lane; c < slab_words / 4; c += kMinLanes) dst[c] = src4[c];
        if (lane == 0) store_key<KB>(blob + L.off_first, b, first);
    }
    if (lane == 0) {
        const uint64_t maxd = m ? (uint64_t)sk[bnd[1]] - first : 0;  // the last anchor is the largest
        const uint32_t ab = byte_width(maxd), sb = byte_width(maxA);
        BlockInfo bi;
        bi.nseg = m;
        bi.seg_bytes = (uint32_t)(a16(2ull * m) + a16((uint64_t)ab * m) + a16((uint64_t)sb * m));
        bi.nkeys = nb;
        bi.ab = (uint8_t)ab;
        bi.sb = (uint8_t)sb;
        bi.pad = 0;
        ws.blk[b] = bi;
    }
}

template <int KB>
__global__ __launch_bounds__(kMinLanes) void fit_min_kernel(const void* __restrict__ keys, Layout L,
                                                             uint8_t* __restrict__ blob, Workspace ws,
                                                             uint32_t* __restrict__ flags, uint64_t blk0)
{
    fit_min_block<KB, false>(keys, L, blob, ws, flags, blk0 + blockIdx.x);  // the launcher keeps b < nblocks
}

// ---------------------------------------------------------------------------
// Optimal fit (LC_FIT_OPT): fixed-point lines with a free intercept, the
// class of the optimal eps-PLA of Sec. II-A.  Segment [s, e) holds a line
// floor((C + A d) / 2^F) with integers A >= 0 and C >= first * 2^F exactly
// when every pair i < j of its keys has
//   ceil((Lo_j - Up_i) / (j - i)) <= A <= floor((Up_j - Lo_i) / (j - i)),
//   Lo_i = (K[i] - eps) 2^F (Lo_s raised to max(K[s] - eps, first) 2^F),
//   Up_i = (K[i] + eps + 1) 2^F - 1,
// and K[e-1] - K[s] + 2 eps + 1 < 2^(64 - F) (the cap: A d + (C mod 2^F)
// stays below 2^64).  Key e adds the pairs (i, e).  The largest new lower
// bound is the steepest line from (e, Lo_e) back to a point (i, Up_i); it
// touches the lower convex hull of those points (all of them lie on or above
// it), and the smallest new upper bound touches the upper hull of the points
// (i, Lo_i) -- O'Rourke's observation.  So each key scans the vertices of two
// hulls of (i, K[i]) (the upper one with the raised start), one vertex per
// lane and a wave max / min, instead of every earlier key.  The hulls are
// kept in LDS as index stacks; their updates are wave-uniform, with exact
// 128-bit cross products.  A sub-segment of a feasible segment is feasible
// (the intercept moved to a later start only grows, as A >= 0), so growing
// each segment as far as it goes gives the fewest segments.  Stored: A =
// floor((lo + hi) / 2) of the final slope interval (0 for one key), C = the
// midpoint of that A's feasible intercepts, anchor delta = floor(C / 2^F) -
// first (mod 2^64), fraction = C mod 2^F.  One wave per block, sequential
// over the block's keys.
// LDS: keys KT[B] | slab u32[res_stride / 4 + 4] | lower hull u16[B] | upper hull u16[B].
// Block b of a list (keys, L, blob slot, workspace of the list); SIZES: the
// size pass, block info only (no records, slab or first key written).
template <int KB, bool SIZES>
__device__ __forceinline__ void fit_opt_block(const void* __restrict__ keys, const Layout L,
                                              uint8_t* __restrict__ blob, const Workspace& ws,
                                              uint32_t* __restrict__ flags, uint64_t b)
{
    using KT = typename std::conditional<KB == 4, uint32_t, uint64_t>::type;
    using u128 = unsigned __int128;
    using i128 = __int128;
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t B = 1u << L.log2b;
    const uint32_t lane = threadIdx.x;
    const uint64_t base = b << L.log2b;
    const uint32_t nb = (L.n - base) < B ? (uint32_t)(L.n - base) : B;  // >= 1
    const KT* Kg = reinterpret_cast<const KT*>(keys) + base;

    KT* sk = reinterpret_cast<KT*>(smem);
    uint32_t* s_slab = reinterpret_cast<uint32_t*>(smem + KB * B);
    const uint32_t slab_words = (uint32_t)(L.res_stride / 4);
    uint16_t* hU = reinterpret_cast<uint16_t*>(smem + KB * B + L.res_stride + 16);  // lower hull
    uint16_t* hL = hU + B;                                                          // upper hull

    bool unsorted = false;
    for (uint32_t j = lane; j < nb; j += 64) {
        const KT k = Kg[j];
        const KT prev = j ? Kg[j - 1] : (b ? Kg[-1] : KT(0));
        unsorted |= k < prev;
        sk[j] = k;
    }
    for (uint32_t i = lane; i < slab_words + 4; i += 64) s_slab[i] = 0;
    if (__ballot(unsorted) != 0 && lane == 0) atomicOr(flags, kFlagUnsorted);
    __syncthreads();

    const uint64_t eps = L.eps, two_e1 = 2 * eps + 1;
    const uint32_t F = L.F, w = L.w;
    const uint64_t wmask = (1ull << w) - 1;
    const uint64_t fmask = (1ull << F) - 1;
    // key e joins only while K[e] - K[s] < lim, i.e. K[e] - K[s] + 2 eps + 1 < 2^(64 - F)
    const uint64_t lim = F == 0 ? ~0ull - 2 * eps : (1ull << (64 - F)) - two_e1;
    const uint64_t first = (uint64_t)sk[0];
    const uint64_t span = (uint64_t)sk[nb - 1] - first;
    // every numerator below is at most (span + 2 eps + 1) 2^F
    const bool fast = span < (1ull << 50) && fast_division_ok(span, 2 * eps, F);
    // hull cross products y (h - h') with y < 2^50 and index differences
    // < 2^13: each product below 2^63 and the sums below 2^64 in u64
    const bool narrow = span < (1ull << 50);

    uint32_t nseg = 0;
    uint64_t maxA = 0, maxd = 0;
    uint32_t s = 0;
    while (s < nb) {
        const uint64_t Ks = (uint64_t)sk[s];
        // the raised start: Lo_s = (K[s] - eps + r) 2^F with r = max(0, first - (K[s] - eps))
        const uint64_t r = Ks - first >= eps ? 0 : eps - (Ks - first);
        // y of hull point i relative to K[s] (the raise only on the upper hull's start)
        auto yU = [&](uint32_t i) -> uint64_t { return (uint64_t)sk[i] - Ks; };
        auto yL = [&](uint32_t i) -> uint64_t { return i == s ? r : (uint64_t)sk[i] - Ks; };
        uint32_t nU = 1, nL = 1;
        hU[0] = (uint16_t)s;  // every lane, as below
        hL[0] = (uint16_t)s;
        __builtin_amdgcn_wave_barrier();
        uint64_t lo = 0, hi = ~0ull;
        uint32_t e = s + 1;
        for (; e < nb; e++) {
            const uint64_t Ke = (uint64_t)sk[e];
            if (Ke - Ks >= lim) break;
            uint64_t cl = 0, ch = ~0ull;
            for (uint32_t v = lane; v < nU; v += 64) {
                // ceil(((K[e] - K[i] - 2 eps - 1) 2^F + 1) / m), positive only when K[e] - K[i] > 2 eps
                const uint32_t i = hU[v];
                const uint64_t Di = Ke - (uint64_t)sk[i];
                if (Di >= two_e1) {
                    const uint32_t m = e - i;
                    const uint64_t q = div_pick(fast, (Di - two_e1) << F, m, recip(m)) + 1;
                    cl = q > cl ? q : cl;
                }
            }
            for (uint32_t v = lane; v < nL; v += 64) {
                // floor(((K[e] + eps + 1 - Lo_j / 2^F) 2^F - 1) / m)
                const uint32_t j = hL[v];
                const uint32_t m = e - j;
                const uint64_t Y = (Ke - (uint64_t)sk[j]) + two_e1 - (j == s ? r : 0);
                const uint64_t q = div_pick(fast, (Y << F) - 1, m, recip(m));
                ch = q < ch ? q : ch;
            }
            cl = wave_max64(cl);
            ch = wave_min64(ch);
            const uint64_t nlo = cl > lo ? cl : lo, nhi = ch < hi ? ch : hi;
            if (nlo > nhi) break;
            lo = nlo;
            hi = nhi;
            // push e on both hulls; a vertex h1 after h2 stays when it lies
            // strictly below (lower hull) / above (upper hull) the line h2 -> e:
            //   (y1 - y2)(e - h2) vs (ye - y2)(h1 - h2), rearranged so every
            //   term is non-negative: y1 (e - h2) + y2 (h1 - h2) vs ye (h1 - h2) + y2 (e - h2)
            const uint64_t ye = Ke - Ks;
            // sign of y1 (e - h2) + y2 (h1 - h2) - ye (h1 - h2) - y2 (e - h2):
            // -1, 0 or 1, in u64 when the block is narrow, else in u128
            auto turn = [&](uint64_t y1, uint64_t y2, uint32_t h1, uint32_t h2) -> int {
                if (narrow) {
                    const uint64_t l = y1 * (e - h2) + y2 * (h1 - h2), r_ = ye * (h1 - h2) + y2 * (e - h2);
                    return l < r_ ? -1 : l > r_ ? 1 : 0;
                }
                const u128 l = (u128)y1 * (e - h2) + (u128)y2 * (h1 - h2);
                const u128 r_ = (u128)ye * (h1 - h2) + (u128)y2 * (e - h2);
                return l < r_ ? -1 : l > r_ ? 1 : 0;
            };
            while (nU >= 2) {
                const uint32_t h1 = hU[nU - 1], h2 = hU[nU - 2];
                if (turn(yU(h1), yU(h2), h1, h2) < 0) break;
                nU--;
            }
            while (nL >= 2) {
                const uint32_t h1 = hL[nL - 1], h2 = hL[nL - 2];
                if (turn(yL(h1), yL(h2), h1, h2) > 0) break;
                nL--;
            }
            // every lane writes the same entries, so each lane's later reads
            // follow its own write in program order (one wave per workgroup:
            // no barrier needed, only the compiler must keep the order)
            __builtin_amdgcn_wave_barrier();
            hU[nU] = (uint16_t)e;
            hL[nL] = (uint16_t)e;
            nU++;
            nL++;
            __builtin_amdgcn_wave_barrier();
        }
        // slope, then the intercept interval [g, h] of that slope, relative to
        // Lo_s = (K[s] - eps + r) 2^F: g' = max(0, max_j (y_j - r) 2^F - A d_j),
        // h' = min_j (y_j + 2 eps + 1 - r) 2^F - 1 - A d_j  (>= g' >= 0)
        const uint64_t A = e > s + 1 ? lo + (hi - lo) / 2 : 0;
        uint64_t gp = 0, hp = ~0ull;
        for (uint32_t j = s + lane; j < e; j += 64) {
            const uint64_t y = (uint64_t)sk[j] - Ks;
            const i128 Ad = (i128)((u128)A * (j - s));
            const i128 scale = (i128)1 << F;  // multiply: y - r may be negative
            const i128 g = j == s ? (i128)0 : ((i128)y - (i128)r) * scale - Ad;
            const i128 h = ((i128)y + (i128)two_e1 - (i128)r) * scale - 1 - Ad;
            const uint64_t gu = g > 0 ? (uint64_t)g : 0;
            const uint64_t hu = h > 0 ? (uint64_t)h : 0;
            gp = gu > gp ? gu : gp;
            hp = hu < hp ? hu : hp;
        }
        gp = wave_max64(gp);
        hp = wave_min64(hp);
        const uint64_t Cp = gp + (hp - gp) / 2;
        const uint64_t c_hi = (Ks - eps + r) + (Cp >> F);  // floor(C / 2^F), modulo 2^64
        const uint64_t frac = Cp & fmask;
        const uint64_t delta = c_hi - first;
        if (lane == 0 && !SIZES) {
            ws.seg_start[base + nseg] = (uint16_t)s;
            ws.seg_delta[base + nseg] = delta;
            ws.seg_A[base + nseg] = A;
            ws.seg_frac[base + nseg] = (uint32_t)frac;
        }
        if (w != 0 && !SIZES) {
            for (uint32_t j = s + lane; j < e; j += 64) {
                const uint64_t pred = c_hi + ((A * (uint64_t)(j - s) + frac) >> F);
                const uint64_t code = ((uint64_t)sk[j] - pred + eps) & wmask;
                const uint32_t bitpos = j * w;
                const uint32_t wd = bitpos >> 5, sh = bitpos & 31;
                const uint64_t v = code << sh;
                atomicOr(&s_slab[wd], (uint32_t)v);
                if (sh + w > 32) atomicOr(&s_slab[wd + 1], (uint32_t)(v >> 32));
            }
        }
        maxA = A > maxA ? A : maxA;
        maxd = delta > maxd ? delta : maxd;
        nseg++;
        s = e;
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    if (!SIZES) {
        uint4* dst = reinterpret_cast<uint4*>(blob + L.off_res + b * L.res_stride);
        const uint4* src4 = reinterpret_cast<const uint4*>(s_slab);
        for (uint32_t c = lane; c < slab_words / 4; c += 64) dst[c] = src4[c];
        if (lane == 0) store_key<KB>(blob + L.off_first, b, first);
    }
    if (lane == 0) {
        const uint32_t ab = byte_width(maxd), sb = byte_width(maxA);
        BlockInfo bi;
        bi.nseg = nseg;
        bi.seg_bytes = (uint32_t)(a16(2ull * nseg) + a16((uint64_t)ab * nseg) + a16((uint64_t)sb * nseg) +
                                  a16((uint64_t)L.fb * nseg));
        bi.nkeys = nb;
        bi.ab = (uint8_t)ab;
        bi.sb = (uint8_t)sb;
        bi.pad = 0;
        ws.blk[b] = bi;
    }
}

template <int KB>
__global__ __launch_bounds__(64) void fit_opt_kernel(const void* __restrict__ keys, Layout L,
                                                     uint8_t* __restrict__ blob, Workspace ws,
                                                     uint32_t* __restrict__ flags, uint64_t blk0)
{
    fit_opt_block<KB, false>(keys, L, blob, ws, flags, blk0 + blockIdx.x);  // the launcher keeps b < nblocks
}

// Sums over tiles of kTileBlocks blocks.
__global__ __launch_bounds__(256) void tile_reduce_kernel(Workspace ws, uint64_t nblocks, uint64_t tile0)
{
    const uint64_t tile = tile0 + blockIdx.x;
    const uint64_t b = tile * kTileBlocks + threadIdx.x;
    uint64_t bytes = 0, nseg = 0;
    if (b < nblocks) {
        const BlockInfo bi = ws.blk[b];
        bytes = bi.seg_bytes;
        nseg = bi.nseg;
    }
    uint64_t tb, tn;
    block_excl_sum<256>(bytes, &tb);
    block_excl_sum<256>(nseg, &tn);
    // maxima of the segment count (low half) and segment-area bytes (high half)
    __shared__ uint64_t s_mx[2][4];
    const uint64_t mn = wave_max(nseg), mb = wave_max(bytes);
    if (lane_id() == 0) {
        s_mx[0][threadIdx.x / 64] = mn;
        s_mx[1][threadIdx.x / 64] = mb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t m0 = 0, m1 = 0;
        for (int k = 0; k < 4; k++) {
            m0 = s_mx[0][k] > m0 ? s_mx[0][k] : m0;
            m1 = s_mx[1][k] > m1 ? s_mx[1][k] : m1;
        }
        TileSum t;
        t.bytes = tb;
        t.nseg = tn;
        t.off = 0;
        t.max_nseg = (uint32_t)m0;
        t.max_seg_bytes = (uint32_t)m1;
        ws.tiles[tile] = t;
    }
}

// The 128-byte header of blob v1 (one thread).
__device__ __forceinline__ void write_header(uint8_t* __restrict__ blob, const Layout& L, uint64_t nseg_total,
                                             uint64_t max_nseg, uint64_t max_area, uint64_t blob_bytes)
{
    uint32_t h[32];
    for (int k = 0; k < 32; k++) h[k] = 0;
    h[0] = kMagic;
    h[1] = kVersion | (L.kb << 16) | (L.log2b << 24);
    h[2] = L.F | (L.w << 8) | (L.flags << 16);
    h[3] = L.eps;
    h[4] = (uint32_t)L.n;            h[5] = (uint32_t)(L.n >> 32);
    h[6] = (uint32_t)L.nblocks;      h[7] = (uint32_t)(L.nblocks >> 32);
    h[8] = (uint32_t)nseg_total;     h[9] = (uint32_t)(nseg_total >> 32);
    h[10] = (uint32_t)max_nseg;      h[11] = (uint32_t)max_area;
    h[12] = (uint32_t)L.off_first;   h[13] = (uint32_t)(L.off_first >> 32);
    h[14] = (uint32_t)L.off_dir;     h[15] = (uint32_t)(L.off_dir >> 32);
    h[16] = (uint32_t)L.off_res;     h[17] = (uint32_t)(L.off_res >> 32);
    h[18] = (uint32_t)L.res_stride;  h[19] = (uint32_t)(L.res_stride >> 32);
    h[20] = (uint32_t)L.off_seg;     h[21] = (uint32_t)(L.off_seg >> 32);
    h[22] = (uint32_t)blob_bytes;    h[23] = (uint32_t)(blob_bytes >> 32);
    uint4* hd = reinterpret_cast<uint4*>(blob);
    for (int k = 0; k < 8; k++) hd[k] = make_uint4(h[4 * k], h[4 * k + 1], h[4 * k + 2], h[4 * k + 3]);
}

// One workgroup: exclusive scan of tile bytes, totals, header, blob size,
// zero padding after first_keys.
__global__ __launch_bounds__(1024) void tile_scan_kernel(Workspace ws, Layout L, uint8_t* __restrict__ blob,
                                                         uint64_t* __restrict__ d_blob_bytes)
{
    const uint64_t ntiles = (L.nblocks + kTileBlocks - 1) / kTileBlocks;
    uint64_t carry = 0, nseg_total = 0, max_nseg = 0, max_area = 0;
    for (uint64_t t0 = 0; t0 < ntiles; t0 += 1024) {
        const uint64_t t = t0 + threadIdx.x;
        uint64_t v = 0, ns = 0, mx = 0, ma = 0;
        if (t < ntiles) {
            const TileSum ts = ws.tiles[t];
            v = ts.bytes;
            ns = ts.nseg;
            mx = ts.max_nseg;
            ma = ts.max_seg_bytes;
        }
        uint64_t tot, tot_ns;
        const uint64_t ex = block_excl_sum<1024>(v, &tot);
        block_excl_sum<1024>(ns, &tot_ns);
        if (t < ntiles) ws.tiles[t].off = carry + ex;
        carry += tot;
        nseg_total += tot_ns;
        __shared__ uint64_t s_mx[2][16];
        const uint64_t wm = wave_max(mx), wa = wave_max(ma);
        if (lane_id() == 0) {
            s_mx[0][threadIdx.x / 64] = wm;
            s_mx[1][threadIdx.x / 64] = wa;
        }
        __syncthreads();
        for (int k = 0; k < 16; k++) {
            max_nseg = s_mx[0][k] > max_nseg ? s_mx[0][k] : max_nseg;
            max_area = s_mx[1][k] > max_area ? s_mx[1][k] : max_area;
        }
        __syncthreads();
    }
    const uint64_t blob_bytes = L.off_seg + carry;
    if (threadIdx.x == 0) {
        write_header(blob, L, nseg_total, max_nseg, max_area, blob_bytes);
        if (d_blob_bytes) *d_blob_bytes = blob_bytes;
    }
    // zero the pad between first_keys and the directory
    const uint64_t fk_end = L.off_first + L.nblocks * L.kb;
    if (threadIdx.x < L.off_dir - fk_end) blob[fk_end + threadIdx.x] = 0;
}

// Directory entries: one thread per block, 256 blocks (one tile) per workgroup.
__global__ __launch_bounds__(256) void dir_emit_kernel(Workspace ws, Layout L, uint8_t* __restrict__ blob,
                                                       uint64_t tile0)
{
    const uint64_t tile = tile0 + blockIdx.x;
    const uint64_t b = tile * kTileBlocks + threadIdx.x;
    BlockInfo bi = {};
    if (b < L.nblocks) bi = ws.blk[b];
    uint64_t tot;
    const uint64_t ex = block_excl_sum<256>(bi.seg_bytes, &tot);
    if (b < L.nblocks) {
        const uint64_t seg_off = L.off_seg + ws.tiles[tile].off + ex;
        const uint32_t w3 = (bi.nkeys - 1) | ((uint32_t)bi.ab << 16) | ((uint32_t)bi.sb << 24);
        reinterpret_cast<uint4*>(blob + L.off_dir)[b] =
            make_uint4((uint32_t)seg_off, (uint32_t)(seg_off >> 32), bi.nseg, w3);
    }
}

// 16 bytes of a little-endian array of `width`-byte values: entries
// [c * 16 / width, (c + 1) * 16 / width), zero past n.
template <typename T>
__device__ __forceinline__ uint4 pack_chunk(const T* vals, uint32_t n, uint32_t c, uint32_t width)
{
    const uint32_t per = 16 / width;
    const uint64_t mask = width == 8 ? ~0ull : ((1ull << (8 * width)) - 1);
    uint64_t lo = 0, hi = 0;
    for (uint32_t k = 0; k < per; k++) {
        const uint32_t idx = c * per + k;
        const uint64_t v = idx < n ? ((uint64_t)vals[idx] & mask) : 0;
        const uint32_t bit = k * width * 8;
        if (bit < 64) lo |= v << bit;
        else hi |= v << (bit - 64);
    }
    return make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
}

// Is directory entry dv of block b consistent with layout L and a blob of
// `bytes` bytes?  Key count as the layout says, 1 <= nseg <= keys, byte
// widths in {1, 2, 4, 8}, the segment area 16-byte aligned inside
// [off_seg, bytes).  Decoders check it before following the offset.
__device__ __forceinline__ bool dir_ok(const uint4& dv, const Layout& L, uint64_t b, uint64_t bytes)
{
    const uint64_t seg_off = dv.x | ((uint64_t)dv.y << 32);
    const uint64_t left = L.n - (b << L.log2b);
    const uint32_t want = left < (1ull << L.log2b) ? (uint32_t)left : (1u << L.log2b);
    const uint32_t nseg = dv.z, nkeys = (dv.w & 0xFFFF) + 1;
    const uint32_t ab = (dv.w >> 16) & 0xFF, sb = dv.w >> 24;
    const bool widths = ab && sb && ab <= 8 && sb <= 8 && !(ab & (ab - 1)) && !(sb & (sb - 1));
    const uint64_t area =
        a16(2ull * nseg) + a16((uint64_t)ab * nseg) + a16((uint64_t)sb * nseg) + a16((uint64_t)L.fb * nseg);
    return nkeys == want && nseg >= 1 && nseg <= nkeys && widths && (seg_off & 15) == 0 && seg_off >= L.off_seg &&
           seg_off <= bytes && area <= bytes - seg_off;
}

constexpr uint32_t kEmitLanes = 16;

// The start, anchor-delta and slope arrays of one segment area (n records
// read from st / dl / sa, LDS or global) packed at byte widths 2, ab and sb
// into 16-byte chunks at out, lanes `lane`, `lane + G`, ... writing; returns
// the first chunk after the slopes.
template <uint32_t G, typename P16, typename P64>
__device__ __forceinline__ uint4* emit_records(P16 st, P64 dl, P64 sa, uint32_t n, uint32_t ab, uint32_t sb,
                                               uint4* __restrict__ out, uint32_t lane)
{
    const uint32_t c_start = (uint32_t)(a16(2ull * n) / 16);
    const uint32_t c_anchor = (uint32_t)(a16((uint64_t)ab * n) / 16);
    const uint32_t c_slope = (uint32_t)(a16((uint64_t)sb * n) / 16);
    for (uint32_t c = lane; c < c_start; c += G) out[c] = pack_chunk(st, n, c, 2);
    out += c_start;
    for (uint32_t c = lane; c < c_anchor; c += G) out[c] = pack_chunk(dl, n, c, ab);
    out += c_anchor;
    for (uint32_t c = lane; c < c_slope; c += G) out[c] = pack_chunk(sa, n, c, sb);
    return out + c_slope;
}

// Segment area of block b (G lanes): the records in the workspace packed at
// the block's widths into 16-byte chunks at the directory's offset.
template <uint32_t G>
__device__ __forceinline__ void emit_block(const Workspace& ws, const Layout& L, uint8_t* __restrict__ blob, uint64_t b)
{
    const uint32_t lane = threadIdx.x % G;
    const uint4 dv = reinterpret_cast<const uint4*>(blob + L.off_dir)[b];
    const uint64_t seg_off = dv.x | ((uint64_t)dv.y << 32);
    const uint32_t n = dv.z;
    const uint32_t ab = (dv.w >> 16) & 0xFF, sb = dv.w >> 24;
    const uint64_t rec = b << L.log2b;
    uint4* out = emit_records<G>(ws.seg_start + rec, ws.seg_delta + rec, ws.seg_A + rec, n, ab, sb,
                                 reinterpret_cast<uint4*>(blob + seg_off), lane);
    if (L.fb) {  // intercept fractions of the optimal fit
        const uint32_t c_frac = (uint32_t)(a16((uint64_t)L.fb * n) / 16);
        for (uint32_t c = lane; c < c_frac; c += G) out[c] = pack_chunk(ws.seg_frac + rec, n, c, L.fb);
    }
}

// Segment areas: kEmitLanes lanes per block, 256 / kEmitLanes blocks per
// workgroup (most blocks need three 16-byte chunks; a whole wave per block
// left most lanes idle).
__global__ __launch_bounds__(256) void seg_emit_kernel(Workspace ws, Layout L, uint8_t* __restrict__ blob,
                                                       uint64_t blk0)
{
    const uint64_t b = blk0 + (uint64_t)blockIdx.x * (256 / kEmitLanes) + threadIdx.x / kEmitLanes;
    if (b >= L.nblocks) return;
    emit_block<kEmitLanes>(ws, L, blob, b);
}

// ---------------------------------------------------------------------------
// Decode
// ---------------------------------------------------------------------------

struct DecodeArgs {
    Layout L;
    uint64_t begin, end;   // key range, global indices
    uint64_t b_first;      // first block of this launch
    uint64_t nblk;         // blocks in this launch
    uint64_t per_xcd;      // ceil(grid / 8): consecutive blocks handled by one XCD
    uint32_t raw_cap;      // LDS bytes for a staged segment area
    uint64_t bytes;        // bytes of the blob (or of its slot): directory offsets must stay inside
    uint32_t* flags;       // where a corrupt directory entry is reported (may be null)
};

// A block's segment area is staged raw in LDS when it is at most
// kSegRawSmall bytes (less when the blob's largest area, a header field, is
// smaller), which keeps ~29 waves resident per CU.  The few larger areas --
// sparse stretches where most segments hold two keys -- are not staged: the
// same wave builds the segment bitmap and decodes the keys reading the model
// arrays from the blob (cached), so no second launch is needed.
constexpr uint32_t kSegRawSmall = 4096;
constexpr uint32_t kTouchGrid = 8192;
constexpr uint64_t kTouchMinBytes = 1ull << 20;  // below this the touch pass costs more than it saves
// 16-byte chunks per lane loaded before the first wait (slab, segment area).
constexpr uint32_t kSlabBatch = 4;
constexpr uint32_t kSegBatch = 4;

__host__ __device__ constexpr uint32_t decode_raw_cap(uint32_t max_seg_bytes, uint32_t cap)
{
    return ((max_seg_bytes < cap ? max_seg_bytes : cap) + 15) & ~15u;
}

__host__ __device__ constexpr uint64_t decode_lds_bytes(uint32_t log2b, uint64_t res_stride, uint32_t raw_cap)
{
    return (uint64_t)raw_cap + 16 + (8ull << log2b) / 32 + res_stride + 16;
}

__device__ __forceinline__ uint32_t wave_incl_sum32(uint32_t v)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

// ---------------------------------------------------------------------------
// Greedy fit with one block per lane (64 blocks per wave), for lists of at
// least kLanesMinBlocks blocks.  The greedy walk consumes exactly one key per
// step -- a key either joins the open segment or closes it and becomes the
// next anchor -- so all 64 walks advance in lockstep over keys 0, 1, 2, ...
// of their blocks: no cross-lane scans, one candidate per lane per step.
// Keys arrive in chunks of kLaneChunk keys per block, loaded coalesced into
// registers one chunk ahead and written to LDS (a row per block, padded
// against bank conflicts).  Slopes follow the same rules as fit_rows; the
// residual codes, which need each segment's final slope, are packed by
// code_pack_kernel from the segment records.
constexpr uint32_t kLaneChunk = 16;
constexpr uint64_t kLanesMinBlocks = 16384;

// Dynamic LDS of a lane-fit launch: the reciprocal table of lanes_fit.
inline size_t lane_fit_lds(uint32_t log2b) { return 8 * ((1ull << log2b) + 2); }

// One lane's block for lanes_fit.
struct LaneBlock {
    uint64_t koff;          // index of the block's first key in the key array
    uint32_t nb;            // keys in the block; 0: the lane has no block
    bool has_prev;          // a key of the same list precedes the block (order check)
    uint64_t eps;           // the block's error bound
    uint16_t* st;           // the block's segment records (RECORDS only)
    uint64_t* dl;
    uint64_t* sa;
    BlockInfo* info;        // where the block's info goes (when nb > 0)
    uint8_t* first_dst;     // the block's first_keys slot (RECORDS only)
};

// The walk of lanes_fit.  Keys arrive in chunks of kLaneChunk keys per
// block, loaded coalesced into registers one chunk ahead and staged through
// a padded LDS tile; each lane reads its chunk into registers before walking
// it.  Loads are unconditional unless some lane of the wave has no block or
// a block reaching past keys_end (then a part past its block's end is loaded
// key by key or not at all): a branch around a load would make the compiler
// wait for every load at the join.  Reading past a block's end but before
// keys_end only reads keys the walk ignores.  A block may start at any
// key-width-aligned address (a batch's lists start anywhere); the 16-byte
// global loads need only dword alignment on this hardware.  Every key address
// is the kernel's key pointer plus an offset (never a pointer rebuilt from an
// integer), so the loads stay global loads: a flat load would also count
// against the LDS wait counter and stall every LDS read behind the chunk
// loads in flight.
template <int KB, bool RECORDS>
__device__ __forceinline__ void lanes_fit(const LaneBlock& in, const void* __restrict__ keys, uint64_t nkeys,
                                          uint32_t log2b, uint32_t F, uint32_t* __restrict__ flags)
{
    using KT = typename std::conditional<KB == 4, uint32_t, uint64_t>::type;
    constexpr uint32_t kPitch = kLaneChunk + 1;        // keys per LDS row
    constexpr uint32_t kParts = kLaneChunk * KB / 16;  // 16-byte loads per block and chunk
    constexpr uint32_t kLoads = kParts;                // loads per lane and chunk (64 blocks per wave)
    constexpr uint32_t kPer = 16 / KB;                 // keys per load
    __shared__ KT s_keys[2][64 * kPitch];
    // 1 / d for d = 0 .. B + 1 (entry 0 unused), from the launch's dynamic LDS
    // (lane_fit_lds bytes): the fast walk reads the next key's reciprocal
    // instead of computing it
    extern __shared__ __align__(16) double s_inv[];

    const uint32_t lane = threadIdx.x;
    const uint32_t B = 1u << log2b;
    const uint32_t nb = in.nb;
    for (uint32_t i = lane; i <= B + 1; i += 64) s_inv[i] = 1.0 / (double)(i > 0 ? i : 1u);  // correctly rounded
    const KT* K0 = reinterpret_cast<const KT*>(keys);
    const KT* Kb = K0 + in.koff;
    const uint64_t kend = nkeys;  // key index bound of every load
    const uint64_t eps = in.eps;
    const uint64_t lim = F == 0 ? (~0ull - eps) : ((1ull << (64 - F)) - eps - 1);
    const uint64_t first = nb ? (uint64_t)Kb[0] : 0;
    // one-round divisions when every block of the wave allows them (a wrapped span does not)
    const bool fast = __ballot(!fast_division_ok(nb ? (uint64_t)Kb[nb - 1] - first : 0, eps, F)) == 0;
    const bool careful = __ballot(nb == 0 || in.koff + B > kend) != 0;  // wave-uniform
    const bool full = __ballot(nb != B) == 0;  // every lane walks a whole block (wave-uniform)

    // the blocks this lane loads parts of, and their key counts (fixed for the walk)
    uint64_t qoff[kLoads];
    uint32_t qn[kLoads];
#pragma unroll
    for (uint32_t i = 0; i < kLoads; i++) {
        const uint32_t q = (i * 64 + lane) / kParts;
        qoff[i] = (uint64_t)__shfl((unsigned long long)in.koff, q, 64);
        qn[i] = (uint32_t)__shfl((int)nb, q, 64);
    }
    uint4 pre[kLoads];
    auto load_chunk = [&](uint32_t c) {
        if (!careful) {  // one branch per chunk around a straight run of loads, all in flight together
#pragma unroll
            for (uint32_t i = 0; i < kLoads; i++) {
                const uint32_t p = (i * 64 + lane) % kParts;
                pre[i] = *reinterpret_cast<const uint4*>(K0 + qoff[i] + c * kLaneChunk + p * kPer);
            }
            return;
        }
#pragma unroll
        for (uint32_t i = 0; i < kLoads; i++) {
            const uint32_t p = (i * 64 + lane) % kParts;
            const KT* bq = K0 + qoff[i];
            const uint32_t j0 = c * kLaneChunk + p * kPer;
            const uint32_t nq = qn[i];
            uint4 v = make_uint4(0, 0, 0, 0);
            if (j0 + kPer <= nq && qoff[i] + j0 + kPer <= kend) {
                v = *reinterpret_cast<const uint4*>(bq + j0);
            } else if (j0 < nq) {
                KT tmp[kPer] = {};
                for (uint32_t u = 0; u < kPer && j0 + u < nq; u++) tmp[u] = bq[j0 + u];
                __builtin_memcpy(&v, tmp, 16);
            }
            pre[i] = v;
        }
    };
    auto store_chunk = [&](uint32_t buf) {
#pragma unroll
        for (uint32_t i = 0; i < kLoads; i++) {
            const uint32_t f = i * 64 + lane, q = f / kParts, p = f % kParts;
            KT v[kPer];
            __builtin_memcpy(v, &pre[i], 16);
#pragma unroll
            for (uint32_t u = 0; u < kPer; u++) s_keys[buf][q * kPitch + p * kPer + u] = v[u];
        }
    };

    uint32_t s = 0, nseg = 0;
    uint64_t Ka = first, P = 0, H = ~0ull, maxA = 0, maxd = 0;
    double inv = 1.0;  // recip(d) for the next key, d = its distance from the anchor
    uint64_t M = ~0ull;                      // the slow path's M
    const double epsf = (double)eps, scf = (double)(1ull << F);
    uint64_t prev = (nb && in.has_prev) ? (uint64_t)Kb[-1] : 0;
    bool unsorted = false;
    uint64_t uns_b = 0;  // ballots of order violations seen by the fast path

    // closes segment [s, e) with slope interval (Pc, Hc) (P encoding: 1 + the
    // largest non-negative lower end, 0 while there is none); when every
    // lower end is negative, lo = -Mc with Mc the running minimum of
    // floor((eps - D) 2^F / d) over the segment's keys, kept by the walk
    auto close = [&](uint32_t e, uint64_t Pc, uint64_t Hc, uint64_t Mc) {
        uint64_t A = 0;
        if (e > s + 1) {
            if (Pc != 0) {
                const uint64_t lo = Pc - 1;
                A = lo + (Hc - lo) / 2;
            } else {
                A = Hc >= Mc ? (Hc - Mc) / 2 : 0;
            }
        }
        if (RECORDS) {
            in.st[nseg] = (uint16_t)s;
            in.dl[nseg] = Ka - first;
            in.sa[nseg] = A;
        }
        nseg++;
        maxA = A > maxA ? A : maxA;
        maxd = Ka - first;  // anchors grow with the segment index
    };

    // Fast path, exact FP64 arithmetic (every numerator is below 2^49).  For
    // key e at distance d = e - s from the anchor s, with D = K[e] - K[s]:
    //   lower end ceil((D - eps) 2^F / d)            = floor(xl / d), xl = D 2^F - eps 2^F + (d - 1) / 2
    //   upper end floor(((D + eps + 1) 2^F - 1) / d) = floor(xh / d), xh = D 2^F + (eps + 1) 2^F - 1 - (d - 1) / 2
    // using floor(y / d) = round((y + 1/2 - d/2) / d) for integers y (and the
    // ceiling as the floor of y + d - 1): that quotient lies at least 1/(2d)
    // inside its rounding interval, and with |y| < 2^49 and 1/d correctly
    // rounded the product errs by at most 1/(16d), so one FMA into the
    // mantissa of 1.5 * 2^52 yields the exact integer, with no remainder
    // correction.  The bounds stay in that offset domain (Lf = kRound +
    // largest lower end, Hf = kRound + smallest upper end); only max, min and
    // compares touch them.  xl and xh split into a per-key term Pk = K' 2^F +
    // e/2 (resp. Qk = K' 2^F - e/2, K' = K[e] - K[0]) and a per-segment term
    // Ca = -eps 2^F - 1/2 - Pk(s) (resp. Cb = (eps + 1) 2^F - 1/2 - Qk(s)),
    // so a step is two adds, two FMAs, a max, a min and a compare.  A closed
    // segment's slope is max(0, Lf + floor((Hf - Lf) / 2)) in real terms: the
    // midpoint of [Lf, Hf], which is also the slow path's (P, H, M) rule.
    // No bound yet: only the high word of a reset bound is set, which puts it
    // beyond every real bound whatever its low word holds.
    constexpr uint32_t kLoResetHi = 0xC3F00000u, kHiResetHi = 0x43F00000u;  // -2^64 .. -2^65, 2^64 .. 2^65
    constexpr double kRound = 6755399441055744.0;  // 1.5 * 2^52: FMA into it rounds to an integer
    constexpr double kTwo52 = 4503599627370496.0;
    const double epsLo = epsf * scf, epsHi = (epsf + 1.0) * scf - 1.0;
    const double cLo = -epsLo - 0.5, cHi = epsHi + 0.5;
    const double m52 = -kTwo52 * scf;  // K' 2^F = fma(2^52 + K', 2^F, -2^52 2^F), exactly
    auto with_hi = [](double v, uint32_t hi) {
        return __longlong_as_double((long long)(((uint64_t)hi << 32) | (uint32_t)__double_as_longlong(v)));
    };
    double Lf = with_hi(0.0, kLoResetHi), Hf = with_hi(0.0, kHiResetHi), Ca = cLo, Cb = cHi;
    double maxAf = 0.0;
    uint64_t Kadu = 0;  // K' of the open segment's anchor
    // LDS byte address of s_inv[d + 1], d = the distance of the current key
    // from its anchor: the reciprocal the next key needs if this one joins
    uint32_t inv_two = (uint32_t)(uintptr_t)(s_inv + 2);
    asm("" : "+v"(inv_two));  // kept in a register, not rebuilt at every step
    uint32_t ib = inv_two;
    auto to_u64 = [](double v) {  // an exact integer below 2^52
        return (uint64_t)__double_as_longlong(v + kTwo52) & 0x000FFFFFFFFFFFFFull;
    };
    // offset-domain bounds -> slope; a block's last segment may hold its
    // anchor only (bounds still reset: slope 0), every other closed segment
    // holds two keys or more (a key one step from its anchor never closes one)
    auto close_f = [&](bool last) {
        double A = vmax_f64(0.0, (Lf - kRound) + __builtin_floor((Hf - Lf) * 0.5));
        if (last) A = Lf < 2251799813685248.0 ? 0.0 : A;
        if (RECORDS) {
            in.st[nseg] = (uint16_t)s;
            in.dl[nseg] = Kadu;
            in.sa[nseg] = to_u64(A);
        }
        nseg++;
        maxAf = vmax_f64(maxAf, A);
    };
    // one key of the fast walk: e = its index (> 0), Pk / Qk its terms,
    // kdu = K' as an integer
    auto step_f = [&](uint32_t e, double Pk, double Qk, uint64_t kdu) {
        const double inv_next = *reinterpret_cast<const __attribute__((address_space(3))) double*>(ib);
        const double ql = __builtin_fma(Pk + Ca, inv, kRound);
        const double qh = __builtin_fma(Qk + Cb, inv, kRound);
        const double Ln = vmax_f64(Lf, ql), Hn = vmin_f64(Hf, qh);
        const bool fail = Ln > Hn;  // the key closes the segment
        const uint64_t m = __builtin_amdgcn_ballot_w64(fail);
        if (fail) {
            close_f(false);
            Ca = cLo - Pk;
            Cb = cHi - Qk;
            s = e;
            Kadu = kdu;
        }
        Lf = with_hi(Ln, sel_u32(m, kLoResetHi, (uint32_t)(__double_as_longlong(Ln) >> 32)));
        Hf = with_hi(Hn, sel_u32(m, kHiResetHi, (uint32_t)(__double_as_longlong(Hn) >> 32)));
        inv = sel_f64(m, 1.0, inv_next);
        ib = sel_u32(m, inv_two, ib + 8);
    };

    const uint32_t nchunks = B / kLaneChunk;
    load_chunk(0);
    store_chunk(0);
    __syncthreads();
    for (uint32_t c = 0; c < nchunks; c++) {
        if (c + 1 < nchunks) load_chunk(c + 1);
        // the lane's kLaneChunk keys of this chunk, all read before the walk
        // (no LDS latency inside the dependent step chain)
        const KT* row = &s_keys[c & 1][lane * kPitch];
        uint64_t kc[kLaneChunk];
#pragma unroll
        for (uint32_t t = 0; t < kLaneChunk; t++) kc[t] = row[t];
        if (fast) {
            // order check and the per-key terms first: independent of the walk
            const double hc = (double)(c * (kLaneChunk / 2));  // e / 2 at t = 0
            double X[kLaneChunk];  // K' 2^F
#pragma unroll
            for (uint32_t t = 0; t < kLaneChunk; t++) {
                const uint32_t e = c * kLaneChunk + t;
                const bool valid = full ? true : e < nb;
                uns_b |= __ballot(valid && kc[t] < prev);
                prev = valid ? kc[t] : prev;
                X[t] = __builtin_fma(__longlong_as_double((long long)(0x4330000000000000ull | (kc[t] - first))), scf,
                                     m52);
            }
            if (full) {
#pragma unroll
                for (uint32_t t = 0; t < kLaneChunk; t++) {
                    const uint32_t e = c * kLaneChunk + t;
                    const double h = hc + 0.5 * t;
                    if (e > 0) step_f(e, X[t] + h, X[t] - h, kc[t] - first);
                }
            } else {
#pragma unroll
                for (uint32_t t = 0; t < kLaneChunk; t++) {
                    const uint32_t e = c * kLaneChunk + t;
                    const double h = hc + 0.5 * t;
                    if (e > 0 && e < nb) step_f(e, X[t] + h, X[t] - h, kc[t] - first);
                }
            }
        } else {
#pragma unroll
            for (uint32_t t = 0; t < kLaneChunk; t++) {
                const uint32_t e = c * kLaneChunk + t;
                const uint64_t key = kc[t];
                if (e < nb) {
                    unsorted |= key < prev;
                    prev = key;
                    if (e > 0) {
                        const uint32_t d = e - s;
                        const double inv_next = recip(d + 1);
                        const uint64_t D = key - Ka;
                        bool fail = D >= lim;
                        uint64_t Pn = P, Hn = H, Mn = M;
                        if (!fail) {
                            // one quotient of |D - eps| 2^F: the lower end, or the M term
                            const bool up = D >= eps;
                            uint32_t rem;
                            const uint64_t q = div_small((up ? D - eps : eps - D) << F, d, inv, &rem);
                            if (up) {
                                const uint64_t pp = q + (rem != 0) + 1;  // 1 + ceil((D - eps) 2^F / d)
                                Pn = pp > P ? pp : P;
                            } else {
                                Mn = q < M ? q : M;  // floor((eps - D) 2^F / d)
                            }
                            const uint64_t h = div_small(((D + eps + 1) << F) - 1, d, inv);
                            Hn = h < H ? h : H;
                            fail = Pn != 0 && Pn - 1 > Hn;
                        }
                        if (fail) {
                            close(e, P, H, M);
                            s = e;
                            Ka = key;
                            P = 0;
                            H = ~0ull;
                            M = ~0ull;
                            inv = 1.0;
                        } else {
                            P = Pn;
                            H = Hn;
                            M = Mn;
                            inv = inv_next;
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (c + 1 < nchunks) store_chunk((c + 1) & 1);
        __syncthreads();
    }
    if (nb) {
        if (fast) {
            close_f(true);
            maxA = to_u64(maxAf);
            maxd = Kadu;
        } else {
            close(nb, P, H, M);
        }
    }
    if ((__ballot(unsorted) | uns_b) != 0 && lane == 0) atomicOr(flags, kFlagUnsorted);
    if (nb) {
        if (RECORDS) {
            if (KB == 4)
                *reinterpret_cast<uint32_t*>(in.first_dst) = (uint32_t)first;
            else
                *reinterpret_cast<uint64_t*>(in.first_dst) = first;
        }
        const uint32_t ab = byte_width(maxd), sb = byte_width(maxA);
        BlockInfo bi;
        bi.nseg = nseg;
        bi.seg_bytes = (uint32_t)(a16(2ull * nseg) + a16((uint64_t)ab * nseg) + a16((uint64_t)sb * nseg));
        bi.nkeys = nb;
        bi.ab = (uint8_t)ab;
        bi.sb = (uint8_t)sb;
        bi.pad = 0;
        *in.info = bi;
    }
}

// Greedy fit with one block per lane (64 blocks per wave), for lists of at
// least kLanesMinBlocks blocks.  The greedy walk consumes exactly one key per
// step -- a key either joins the open segment or closes it and becomes the
// next anchor -- so all 64 walks advance in lockstep over keys 0, 1, 2, ...
// of their blocks: no cross-lane scans, one candidate per lane per step.
// Slopes follow the same rules as fit_rows; the residual codes, which need
// each segment's final slope, are packed by code_pack_kernel from the
// segment records.
template <int KB>
__global__ __launch_bounds__(64) void fit_lanes_kernel(const void* __restrict__ keys, Layout L,
                                                        uint8_t* __restrict__ blob, Workspace ws,
                                                        uint32_t* __restrict__ flags, uint64_t blk0)
{
    const uint64_t b = blk0 + (uint64_t)blockIdx.x * 64 + threadIdx.x;
    const bool has = b < L.nblocks;
    const uint32_t B = 1u << L.log2b;
    LaneBlock in;
    in.nb = has ? ((L.n - (b << L.log2b)) < B ? (uint32_t)(L.n - (b << L.log2b)) : B) : 0u;
    in.koff = has ? (b << L.log2b) : 0;
    in.has_prev = b > 0;
    in.eps = L.eps;
    const uint64_t rec = has ? (b << L.log2b) : 0;
    in.st = ws.seg_start + rec;
    in.dl = ws.seg_delta + rec;
    in.sa = ws.seg_A + rec;
    in.info = ws.blk + (has ? b : 0);
    in.first_dst = blob + L.off_first + (has ? b : 0) * KB;
    lanes_fit<KB, true>(in, keys, L.n, L.log2b, L.F, flags);
}

// Residual codes of one block from its segment records (one wave per block):
// the records' starts -> LDS bitmap with per-word prefix counts, so key j's
// segment is the number of starts <= j, minus one; code = K[j] - pred + eps
// packed LSB-first into the LDS slab, then copied to the blob.  Records of
// blocks with at most kCodeSegCap segments are staged in LDS; larger ones
// are read from the workspace.  Keys are loaded 16 per lane ahead of use.
// LDS: bitmap u32[B / 32] | prefix u32[B / 32] | slab u32[res_stride / 4 + 4] |
// deltas u64[cap] | slopes u64[cap] | starts u16[cap].
constexpr uint32_t kCodeSegCap = 256;

inline size_t code_pack_lds(uint32_t log2b, uint64_t res_stride)
{
    return 8 * ((1ull << log2b) >> 5) + res_stride + 16 + 18 * kCodeSegCap;
}

template <int KB>
__device__ __forceinline__ void code_pack_block(const void* __restrict__ keys, const BlockInfo& bi,
                                                const uint16_t* __restrict__ rst, const uint64_t* __restrict__ rdl,
                                                const uint64_t* __restrict__ rsa, uint32_t log2b,
                                                uint64_t res_stride, uint32_t w, uint64_t eps, uint32_t F,
                                                uint8_t* __restrict__ slab_dst, uint4* __restrict__ seg_dst = nullptr,
                                                uint32_t ab = 0, uint32_t sb = 0)
{
    using KT = typename std::conditional<KB == 4, uint32_t, uint64_t>::type;
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t lane = threadIdx.x;
    const uint32_t B = 1u << log2b, nwords = B >> 5;
    const uint32_t nb = bi.nkeys <= B ? bi.nkeys : B, nseg = bi.nseg <= B ? bi.nseg : B;
    const uint32_t slab_words = (uint32_t)(res_stride / 4);
    uint32_t* s_bm = reinterpret_cast<uint32_t*>(smem);
    uint32_t* s_pre = s_bm + nwords;
    uint32_t* s_slab = s_pre + nwords;
    uint64_t* s_delta = reinterpret_cast<uint64_t*>(s_slab + slab_words + 4);  // 16-byte aligned
    uint64_t* s_A = s_delta + kCodeSegCap;
    uint16_t* s_st = reinterpret_cast<uint16_t*>(s_A + kCodeSegCap);
    const KT* K = reinterpret_cast<const KT*>(keys);
    const bool staged = nseg <= kCodeSegCap;
    if (nb == 0) return;

    for (uint32_t x = lane; x < nwords; x += 64) s_bm[x] = 0;
    for (uint32_t x = lane; x < slab_words + 4; x += 64) s_slab[x] = 0;
    __syncthreads();
    const uint32_t smask = B - 1;
    for (uint32_t t = lane; t < nseg; t += 64) {
        const uint32_t st = rst[t] & smask;
        atomicOr(&s_bm[st >> 5], 1u << (st & 31));
        if (staged) {
            s_st[t] = (uint16_t)st;
            s_delta[t] = rdl[t];
            s_A[t] = rsa[t];
        }
    }
    __syncthreads();
    // the block's segment area, when the directory is already written (from
    // the staged copy of the records when there is one)
    if (seg_dst != nullptr) {
        if (staged)
            emit_records<64>(s_st, s_delta, s_A, nseg, ab, sb, seg_dst, lane);
        else
            emit_records<64>(rst, rdl, rsa, nseg, ab, sb, seg_dst, lane);
    }
    uint32_t carry = 0;
    for (uint32_t w0 = 0; w0 < nwords; w0 += 64) {
        const uint32_t x = w0 + lane;
        const uint32_t cnt = x < nwords ? __popc(s_bm[x]) : 0u;
        const uint32_t incl = wave_incl_sum32(cnt);
        if (x < nwords) s_pre[x] = carry + incl - cnt;
        carry += __shfl(incl, 63, 64);
    }
    __syncthreads();

    const uint64_t first = (uint64_t)K[0];
    const uint64_t wmask = (1ull << w) - 1;
    const uint32_t tmax = nseg ? nseg - 1 : 0;
    // one loop per record source, so each read has one address space (a
    // pointer chosen at run time would become a flat load, which waits for
    // every outstanding key load)
    auto pack = [&](auto rd) {
        for (uint32_t j0 = 0; j0 < nb; j0 += 16 * 64) {
            uint64_t kv[16];
#pragma unroll
            for (uint32_t i = 0; i < 16; i++) {  // unconditional (clamped) loads: all 16 in flight
                const uint32_t j = j0 + i * 64 + lane;
                kv[i] = (uint64_t)K[j < nb ? j : nb - 1];
            }
#pragma unroll
            for (uint32_t i = 0; i < 16; i++) {
                const uint32_t j = j0 + i * 64 + lane;
                if (j >= nb) continue;
                const uint32_t wd = j >> 5, bit = j & 31;
                const uint32_t r = s_pre[wd] + __popc(s_bm[wd] & ((2u << bit) - 1u));
                const uint32_t t = r ? (r - 1 < tmax ? r - 1 : tmax) : 0u;  // key 0 always starts segment 0
                uint32_t s;
                uint64_t delta, A;
                rd(t, s, delta, A);
                const uint64_t pred = first + delta + ((A * (uint64_t)(j - s)) >> F);
                const uint64_t code = (kv[i] - pred + eps) & wmask;
                const uint32_t bitpos = j * w;
                const uint32_t wo = bitpos >> 5, sh = bitpos & 31;
                const uint64_t v = code << sh;
                atomicOr(&s_slab[wo], (uint32_t)v);
                if (sh + w > 32) atomicOr(&s_slab[wo + 1], (uint32_t)(v >> 32));
            }
        }
    };
    if (w != 0 && staged)
        pack([&](uint32_t t, uint32_t& s, uint64_t& delta, uint64_t& A) {
            s = s_st[t];
            delta = s_delta[t];
            A = s_A[t];
        });
    else if (w != 0)
        pack([&](uint32_t t, uint32_t& s, uint64_t& delta, uint64_t& A) {
            s = rst[t];
            delta = rdl[t];
            A = rsa[t];
        });
    __syncthreads();
    uint4* dst = reinterpret_cast<uint4*>(slab_dst);
    const uint4* src4 = reinterpret_cast<const uint4*>(s_slab);
    for (uint32_t c = lane; c < slab_words / 4; c += 64) dst[c] = src4[c];
}

// Residual slab and segment area of block b, after the directory is written
// (the area goes to the directory entry's offset, at its byte widths).
template <int KB>
__global__ __launch_bounds__(64) void code_pack_kernel(const void* __restrict__ keys, Layout L,
                                                        uint8_t* __restrict__ blob, Workspace ws, uint64_t blk0)
{
    const uint64_t b = blk0 + blockIdx.x;  // the launcher keeps b < nblocks
    const uint64_t rec = b << L.log2b;
    const uint4 dv = reinterpret_cast<const uint4*>(blob + L.off_dir)[b];
    const uint64_t seg_off = dv.x | ((uint64_t)dv.y << 32);
    code_pack_block<KB>(reinterpret_cast<const uint8_t*>(keys) + rec * KB, ws.blk[b], ws.seg_start + rec,
                        ws.seg_delta + rec, ws.seg_A + rec, L.log2b, L.res_stride, L.w, L.eps, L.F,
                        blob + L.off_res + b * L.res_stride, reinterpret_cast<uint4*>(blob + seg_off),
                        (dv.w >> 16) & 0xFF, dv.w >> 24);
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Per-block decode context.
struct BlockCtx {
    uint64_t first, eps, obase;
    uint32_t F, w, ab, sb, fb, jlo, jhi;
    uint32_t tmax;  // last segment index of the block
    const uint32_t* s_slab;
    const uint32_t* s_bm;
    const uint32_t* s_pre;
};

template <uint32_t W, typename P8>
__device__ __forceinline__ uint64_t load_fixed(P8 base, uint32_t t)
{
    if constexpr (W == 1) return base[t];
    else if constexpr (W == 2) return reinterpret_cast<const uint16_t*>(base)[t];
    else if constexpr (W == 4) return reinterpret_cast<const uint32_t*>(base)[t];
    else return reinterpret_cast<const uint64_t*>(base)[t];
}

// floor(A * d / 2^F) with d < 2^13; a 32 x 32 -> 64-bit product when the
// block's slopes fit in 4 bytes.
template <uint32_t SB>
__device__ __forceinline__ uint64_t slope_term(uint64_t A, uint32_t d, uint32_t F)
{
    if constexpr (SB <= 4) return ((uint64_t)(uint32_t)A * d) >> F;
    else return (A * d) >> F;
}

// Decodes keys [jlo, jhi) of one block whose model arrays (u16 start[],
// anchor-first_key[] of AB bytes, A[] of SB bytes, and with FRAC the
// intercept fractions of c.fb bytes) are read through `start`, `an`, `sl`,
// `fr` -- LDS copies for staged blocks, the blob otherwise.  AB / SB / FB
// are the block's byte widths (0: read at the runtime widths).
//
// F0 (integer slopes, no intercept fractions): key = first - eps + anchor +
// A d + code modulo 2^(8 KB), so u32 keys take 32-bit arithmetic only, u64
// keys one 32 x 32 -> 64 multiply-add when the block's slopes fit 4 bytes,
// and the code comes out of its two slab words by one funnel shift.  Used
// for u32 keys (batch decode of u32 lists 0.52 -> 0.50 ms); for u64 keys it
// measured 2-3 % slower than the general path, which they keep.
template <int KB, bool RANGE, bool CLAMP, uint32_t AB, uint32_t SB, bool FRAC, uint32_t FB = 0, bool F0 = false,
          typename P16, typename P8>
__device__ __forceinline__ void decode_keys(const BlockCtx& c, P16 start, P8 an, P8 sl, P8 fr,
                                            void* __restrict__ out)
{
    static_assert(!(F0 && FRAC), "integer slopes carry no fractions");
    constexpr uint32_t V = 16 / KB;
    const uint32_t lane = lane_id();
    const uint64_t wmask = (1ull << c.w) - 1;  // w <= 32
    const uint32_t wmask32 = (uint32_t)wmask;
    const uint64_t first_e = c.first - c.eps;
    auto anchor_of = [&](uint32_t t) -> uint64_t {
        if constexpr (AB != 0) return load_fixed<AB>(an, t);
        else return load_w(an, t, c.ab);
    };
    auto slope_of = [&](uint32_t t) -> uint64_t {
        if constexpr (SB != 0) return load_fixed<SB>(sl, t);
        else return load_w(sl, t, c.sb);
    };
    auto key_at = [&](uint32_t j, uint32_t t) -> uint64_t {
        // keys past the block end in a block's last group (never stored) may
        // count stray bitmap bits; CLAMP keeps their model reads inside the
        // arrays when those live in global memory
        if constexpr (CLAMP) t = t < c.tmax ? t : c.tmax;
        const uint32_t d = j - start[t];
        if constexpr (F0) {
            const uint32_t bitpos = j * c.w;
            const uint32_t wd = bitpos >> 5;
            const uint32_t code = __builtin_amdgcn_alignbit(c.s_slab[wd + 1], c.s_slab[wd], bitpos & 31) & wmask32;
            if constexpr (KB == 4) {
                return (uint32_t)first_e + (uint32_t)anchor_of(t) + (uint32_t)slope_of(t) * d + code;
            } else if constexpr (SB != 0 && SB <= 4) {
                return first_e + anchor_of(t) + code + (uint64_t)(uint32_t)slope_of(t) * d;
            } else {
                return first_e + anchor_of(t) + code + slope_of(t) * d;
            }
        }
        uint64_t pred;
        if constexpr (FRAC) {  // A d + frac < 2^64 (the optimal fit's cap)
            uint64_t f;
            if constexpr (FB != 0) f = load_fixed<FB>(fr, t);
            else f = load_w(fr, t, c.fb);
            pred = c.first + anchor_of(t) + ((slope_of(t) * d + f) >> c.F);
        } else
            pred = c.first + anchor_of(t) + slope_term<SB == 0 ? 8 : SB>(slope_of(t), d, c.F);
        const uint32_t bitpos = j * c.w;
        const uint32_t wd = bitpos >> 5, sh = bitpos & 31;
        const uint64_t win = (uint64_t)c.s_slab[wd] | ((uint64_t)c.s_slab[wd + 1] << 32);
        return pred + ((win >> sh) & wmask) - c.eps;
    };
    auto seg_of = [&](uint32_t j) {
        const uint32_t bits = c.s_bm[j >> 5];
        return c.s_pre[j >> 5] + __popc(bits & (0xFFFFFFFFu >> (31 - (j & 31)))) - 1;
    };

    // Groups of V keys whose output lands on a 16-byte boundary start at
    // j = j0 (mod V); keys [0, j0) of the block are stored one by one.  A
    // group may straddle two bitmap words when j0 != 0, hence the 64-bit
    // window of the bitmap.
    const uint32_t j0 = (uint32_t)(0 - (reinterpret_cast<uintptr_t>(out) / KB + c.obase)) & (V - 1);
    if (lane < j0 && lane >= c.jlo && lane < c.jhi) store_key<KB>(out, c.obase + lane, key_at(lane, seg_of(lane)));
    if constexpr (F0 && KB == 4) {
        // A lane's groups are 64 V keys apart, a multiple of 32, so the slab
        // word offset and shift of its key g + k, its bit in the bitmap word
        // pair and the prefix mask are the same in every group: computed
        // once, then a group advances by 2 V w slab words and 2 V bitmap
        // words.
        const uint32_t g0 = j0 + lane * V;
        uint32_t wo[V], sh[V];
#pragma unroll
        for (uint32_t k = 0; k < V; k++) {
            const uint32_t bp = (g0 + k) * c.w;
            wo[k] = bp >> 5;
            sh[k] = bp & 31;
        }
        const uint32_t bsh = g0 & 31;
        const uint32_t m0 = 0xFFFFFFFFu >> (31 - bsh);
        const uint32_t fe = (uint32_t)first_e;
        uint32_t sw = 0, wb = g0 >> 5;
        for (uint32_t g = g0; g < c.jhi; g += 64 * V, sw += 2 * V * c.w, wb += 2 * V) {
            if (RANGE && g + V <= c.jlo) continue;
            const uint64_t bits = (uint64_t)c.s_bm[wb] | ((uint64_t)c.s_bm[wb + 1] << 32);
            uint32_t t = c.s_pre[wb] + __popc((uint32_t)bits & m0) - 1;
            uint32_t v[V];
#pragma unroll
            for (uint32_t k = 0; k < V; k++) {
                if (k) t += (uint32_t)(bits >> (bsh + k)) & 1u;
                uint32_t tc = t;
                if constexpr (CLAMP) tc = tc < c.tmax ? tc : c.tmax;
                const uint32_t* sp = c.s_slab + sw + wo[k];
                const uint32_t code = __builtin_amdgcn_alignbit(sp[1], sp[0], sh[k]) & wmask32;
                v[k] = fe + (uint32_t)anchor_of(tc) + (uint32_t)slope_of(tc) * (g + k - start[tc]) + code;
            }
            if (g >= c.jlo && g + V <= c.jhi) {
                __builtin_nontemporal_store(u32x4{v[0], v[1], v[2], v[3]},
                                            reinterpret_cast<u32x4*>(reinterpret_cast<uint8_t*>(out) + (c.obase + g) * KB));
            } else {
#pragma unroll
                for (uint32_t k = 0; k < V; k++)
                    if (g + k >= c.jlo && g + k < c.jhi) store_key<KB>(out, c.obase + g + k, v[k]);
            }
        }
        return;
    }
    for (uint32_t g = j0 + lane * V; g < c.jhi; g += 64 * V) {
        if (RANGE && g + V <= c.jlo) continue;
        const uint32_t wb = g >> 5;
        const uint64_t bits = (uint64_t)c.s_bm[wb] | ((uint64_t)c.s_bm[wb + 1] << 32);
        uint32_t t = c.s_pre[wb] + __popc((uint32_t)bits & (0xFFFFFFFFu >> (31 - (g & 31)))) - 1;
        uint64_t v[V];
#pragma unroll
        for (uint32_t k = 0; k < V; k++) {
            const uint32_t j = g + k;
            if (k) t += (uint32_t)(bits >> (j - (wb << 5))) & 1u;
            v[k] = key_at(j, t);
        }
        if (g >= c.jlo && g + V <= c.jhi) {
            u32x4 q;
            if constexpr (KB == 8) {
                q = u32x4{(uint32_t)v[0], (uint32_t)(v[0] >> 32), (uint32_t)v[1], (uint32_t)(v[1] >> 32)};
            } else {
                q = u32x4{(uint32_t)v[0], (uint32_t)v[1], (uint32_t)v[2], (uint32_t)v[3]};
            }
            __builtin_nontemporal_store(q, reinterpret_cast<u32x4*>(reinterpret_cast<uint8_t*>(out) +
                                                                     (c.obase + g) * KB));
        } else {
#pragma unroll
            for (uint32_t k = 0; k < V; k++)
                if (g + k >= c.jlo && g + k < c.jhi) store_key<KB>(out, c.obase + g + k, v[k]);
        }
    }
}

// Staged blocks: dispatch once per block on the (anchor, slope) widths so the
// per-key loop has no width branches.
template <int KB, bool RANGE, bool CLAMP>
__device__ __forceinline__ void decode_staged(const BlockCtx& c, const uint8_t* s_raw, uint32_t off_an,
                                              uint32_t off_sl, uint32_t off_fr, void* __restrict__ out)
{
    const uint16_t* st = reinterpret_cast<const uint16_t*>(s_raw);
    const uint8_t* an = s_raw + off_an;
    const uint8_t* sl = s_raw + off_sl;
#define LC_DECODE_CASE(A_, S_) \
    case (A_) * 16 + (S_):                                                                      \
        if (KB == 4 && c.F == 0)                                                                \
            decode_keys<KB, RANGE, CLAMP, A_, S_, false, 0, true>(c, st, an, sl, sl, out);      \
        else                                                                                    \
            decode_keys<KB, RANGE, CLAMP, A_, S_, false>(c, st, an, sl, sl, out);               \
        return;
#define LC_DECODE_FRAC4_CASE(A_, S_) \
    case (A_) * 16 + (S_): decode_keys<KB, RANGE, CLAMP, A_, S_, true, 4>(c, st, an, sl, s_raw + off_fr, out); return;
    if (c.fb) {  // blobs of the optimal fit: fixed widths for 4-byte fractions (F > 16)
        if (c.fb == 4) {
            switch (c.ab * 16 + c.sb) {
                LC_DECODE_FRAC4_CASE(1, 1) LC_DECODE_FRAC4_CASE(1, 2) LC_DECODE_FRAC4_CASE(1, 4) LC_DECODE_FRAC4_CASE(1, 8)
                LC_DECODE_FRAC4_CASE(2, 1) LC_DECODE_FRAC4_CASE(2, 2) LC_DECODE_FRAC4_CASE(2, 4) LC_DECODE_FRAC4_CASE(2, 8)
                LC_DECODE_FRAC4_CASE(4, 1) LC_DECODE_FRAC4_CASE(4, 2) LC_DECODE_FRAC4_CASE(4, 4) LC_DECODE_FRAC4_CASE(4, 8)
                LC_DECODE_FRAC4_CASE(8, 1) LC_DECODE_FRAC4_CASE(8, 2) LC_DECODE_FRAC4_CASE(8, 4) LC_DECODE_FRAC4_CASE(8, 8)
                default: break;
            }
        }
        decode_keys<KB, RANGE, CLAMP, 0, 0, true>(c, st, an, sl, s_raw + off_fr, out);
        return;
    }
    switch (c.ab * 16 + c.sb) {
        LC_DECODE_CASE(1, 1) LC_DECODE_CASE(1, 2) LC_DECODE_CASE(1, 4) LC_DECODE_CASE(1, 8)
        LC_DECODE_CASE(2, 1) LC_DECODE_CASE(2, 2) LC_DECODE_CASE(2, 4) LC_DECODE_CASE(2, 8)
        LC_DECODE_CASE(4, 1) LC_DECODE_CASE(4, 2) LC_DECODE_CASE(4, 4) LC_DECODE_CASE(4, 8)
        LC_DECODE_CASE(8, 1) LC_DECODE_CASE(8, 2) LC_DECODE_CASE(8, 4) LC_DECODE_CASE(8, 8)
        default: decode_keys<KB, RANGE, CLAMP, 0, 0, false>(c, st, an, sl, sl, out); return;
    }
#undef LC_DECODE_CASE
#undef LC_DECODE_FRAC4_CASE
}

// Streams bytes [lo, hi) of the blob through the caches (wide coalesced
// reads whose values are discarded), so that the decode that follows finds
// them in the 256 MB on-die cache: its reads form a dependent chain per
// block (directory entry -> segment area), so it is bound by memory latency
// when they come from HBM, while this pass reads at full bandwidth.
__global__ __launch_bounds__(256) void touch_kernel(const uint8_t* __restrict__ blob, uint64_t lo, uint64_t hi)
{
    const uint4* p = reinterpret_cast<const uint4*>(blob + lo);
    const uint64_t n = (hi - lo) / 16;
    uint32_t acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        const uint4 v = p[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    asm volatile("" ::"v"(acc));  // keeps the loads; no instruction is emitted
}

// One wave per block.
//  1. Coalesced 16-byte loads of the residual slab (its address needs only
//     b) and of the raw segment area (once the directory entry is in), all
//     unconditional with clamped chunk indices -- every load stays inside
//     the blob; a slab of width 0 reads the first chunk of the segment areas
//     -- so all are in flight before the first wait; they land in LDS.
//  2. The segment starts become an LDS bitmap with per-word prefix
//     popcounts, so the segment of key j is found in O(1):
//       t = prefix[j / 32] + popcount(bits[j / 32] & mask(j % 32)) - 1.
//  3. Lane l decodes the groups of V = 16 / KB keys starting at
//     j0 + V * (l + 64 i), j0 chosen so that every group's output is
//     16-byte aligned; each store instruction of the wave writes 1 KB of
//     contiguous output (non-temporal: the output is not re-read here).
// APPROX: the model alone (approximate query processing, Sec. III-C): the
// residual slab is not read and every key is its prediction f(i), within
// eps of K[i].
template <int KB, bool RANGE, bool APPROX = false>
__device__ __forceinline__ void decode_block(const uint8_t* __restrict__ blob, const DecodeArgs& a, uint64_t b,
                                             uint32_t raw_cap, void* __restrict__ out)
{
    const Layout& L = a.L;
    const uint32_t lane = threadIdx.x;
    const uint32_t nwords = (1u << L.log2b) >> 5;
    const uint32_t slab_words = (uint32_t)(L.res_stride / 4);
    const uint32_t nch_slab = APPROX ? 0u : slab_words / 4;

    extern __shared__ __align__(16) uint8_t smem[];
    uint8_t* s_raw = smem;                                                 // raw_cap
    uint4* s_trash = reinterpret_cast<uint4*>(smem + raw_cap);             // 16 B
    uint32_t* s_slab = reinterpret_cast<uint32_t*>(smem + raw_cap + 16);   // slab_words + 4
    uint32_t* s_bm = s_slab + slab_words + 4;                              // nwords
    uint32_t* s_pre = s_bm + nwords;                                       // nwords

    const uint32_t last_slab = nch_slab ? nch_slab - 1 : 0u;
    const uint4* g_slab = reinterpret_cast<const uint4*>(blob + L.off_res + b * L.res_stride);
    uint4 fs0 = make_uint4(0, 0, 0, 0), fs1 = fs0, fs2 = fs0, fs3 = fs0;
    if constexpr (!APPROX) {
        fs0 = g_slab[lane < last_slab ? lane : last_slab];
        fs1 = g_slab[lane + 64 < last_slab ? lane + 64 : last_slab];
        fs2 = g_slab[lane + 128 < last_slab ? lane + 128 : last_slab];
        fs3 = g_slab[lane + 192 < last_slab ? lane + 192 : last_slab];
    }

    const uint4 dv = reinterpret_cast<const uint4*>(blob + L.off_dir)[b];
    const uint64_t seg_off = dv.x | ((uint64_t)dv.y << 32);
    const uint32_t nseg = dv.z ? dv.z : 1u;
    const uint32_t nkeys = (dv.w & 0xFFFF) + 1;
    const uint32_t ab = (dv.w >> 16) & 0xFF, sb = dv.w >> 24;
    const uint64_t first = load_key<KB>(blob + L.off_first, b);
    const uint32_t off_an = (uint32_t)a16(2ull * nseg);
    const uint32_t off_sl = off_an + (uint32_t)a16((uint64_t)ab * nseg);
    const uint32_t off_fr = off_sl + (uint32_t)a16((uint64_t)sb * nseg);
    const uint32_t seg_bytes = off_fr + (uint32_t)a16((uint64_t)L.fb * nseg);
    if (!dir_ok(dv, L, b, a.bytes)) {  // corrupt blob: skip the block
        if (a.flags && lane == 0) atomicOr(a.flags, kFlagBadList);
        return;
    }
    const bool staged = seg_bytes <= raw_cap;
    const uint8_t* g_seg = blob + seg_off;

    const uint32_t nch_seg = staged ? seg_bytes / 16 : 0u;
    const uint32_t last_seg = nch_seg ? nch_seg - 1 : 0u;
    const uint4* g_raw = reinterpret_cast<const uint4*>(g_seg);
    const uint4 fg0 = g_raw[lane < last_seg ? lane : last_seg];
    const uint4 fg1 = g_raw[lane + 64 < last_seg ? lane + 64 : last_seg];
    const uint4 fg2 = g_raw[lane + 128 < last_seg ? lane + 128 : last_seg];
    const uint4 fg3 = g_raw[lane + 192 < last_seg ? lane + 192 : last_seg];
    {
        // stores unconditional too (lanes past the end write a trash slot),
        // so the compiler cannot sink each load into its own guarded store
        uint4* ss = reinterpret_cast<uint4*>(s_slab);
        uint4* sr = reinterpret_cast<uint4*>(s_raw);
        *(lane < nch_slab ? ss + lane : s_trash) = fs0;
        *(lane + 64 < nch_slab ? ss + lane + 64 : s_trash) = fs1;
        *(lane + 128 < nch_slab ? ss + lane + 128 : s_trash) = fs2;
        *(lane + 192 < nch_slab ? ss + lane + 192 : s_trash) = fs3;
        *(lane < nch_seg ? sr + lane : s_trash) = fg0;
        *(lane + 64 < nch_seg ? sr + lane + 64 : s_trash) = fg1;
        *(lane + 128 < nch_seg ? sr + lane + 128 : s_trash) = fg2;
        *(lane + 192 < nch_seg ? sr + lane + 192 : s_trash) = fg3;
    }
    for (uint32_t c = lane + 64 * kSegBatch; c < nch_seg; c += 64)  // areas over 4 KB
        reinterpret_cast<uint4*>(s_raw)[c] = g_raw[c];
    for (uint32_t c = lane + 64 * kSlabBatch; c < nch_slab; c += 64)  // slabs over 4 KB
        reinterpret_cast<uint4*>(s_slab)[c] = g_slab[c];
    if (lane < 4) s_slab[slab_words + lane] = 0;
    for (uint32_t w = lane; w < nwords; w += 64) s_bm[w] = 0;
    __syncthreads();

    BlockCtx c;
    c.first = first;
    c.eps = APPROX ? 0 : L.eps;  // with w = 0 the code term vanishes: the key is f(i)
    c.F = L.F;
    c.w = APPROX ? 0 : L.w;
    c.ab = ab;
    c.sb = sb;
    c.fb = L.fb;
    c.s_slab = s_slab;
    c.s_bm = s_bm;
    c.s_pre = s_pre;
    c.tmax = nseg - 1;
    const uint64_t i0 = b << L.log2b;
    c.jlo = 0;
    c.jhi = nkeys;
    c.obase = i0;  // out index of key j is obase + j (mod 2^64)
    if constexpr (RANGE) {
        c.jlo = (uint32_t)((a.begin > i0 ? a.begin : i0) - i0);
        const uint64_t iend = i0 + nkeys < a.end ? i0 + nkeys : a.end;
        c.jhi = (uint32_t)(iend - i0);
        c.obase = i0 - a.begin;
    }
    // segment starts -> LDS bitmap + per-word prefix counts
    auto build_bitmap = [&](const uint16_t* st16) {
        const uint32_t smask = (1u << L.log2b) - 1;
        for (uint32_t t = lane; t < nseg; t += 64) {
            const uint32_t st = st16[t] & smask;
            atomicOr(&s_bm[st >> 5], 1u << (st & 31));
        }
        __syncthreads();
        uint32_t carry = 0;
        for (uint32_t w0 = 0; w0 < nwords; w0 += 64) {
            const uint32_t w = w0 + lane;
            const uint32_t cnt = w < nwords ? __popc(s_bm[w]) : 0u;
            const uint32_t incl = wave_incl_sum32(cnt);
            if (w < nwords) s_pre[w] = carry + incl - cnt;
            carry += __shfl(incl, 63, 64);
        }
        __syncthreads();
    };
    if (!staged) {  // model arrays read from the blob (cached), keys decoded as for staged blocks
        build_bitmap(reinterpret_cast<const uint16_t*>(g_seg));
        decode_staged<KB, RANGE, true>(c, g_seg, off_an, off_sl, off_fr, out);
        return;
    }
    build_bitmap(reinterpret_cast<const uint16_t*>(s_raw));
    decode_staged<KB, RANGE, false>(c, s_raw, off_an, off_sl, off_fr, out);
}

// One wave per block.  Workgroup w runs on XCD w % 8, so blocks are
// assigned XCD-major: each XCD walks a contiguous run of blocks (and of
// directory and segment bytes).
template <int KB, bool RANGE, bool APPROX = false>
__global__ __launch_bounds__(64) void decode_kernel(const uint8_t* __restrict__ blob, DecodeArgs a,
                                                     void* __restrict__ out)
{
    const uint64_t rel = (uint64_t)(blockIdx.x % 8) * a.per_xcd + blockIdx.x / 8;
    if (rel >= a.nblk) return;
    decode_block<KB, RANGE, APPROX>(blob, a, a.b_first + rel, a.raw_cap, out);
}

// Decode with the cache staging in the same launch: the first T
// workgroups stream chunks of kStreamChunk blocks of the launch's blocks
// [b_first, b_first + nblk) (directory entries, slabs, then the segment
// areas found from the chunk's first and last directory entries, checked
// against the layout) through the caches in block order, eight 16-byte
// loads in flight per lane; the remaining workgroups decode one block
// each, XCD-major, as decode_kernel (RANGE: the keys of [begin, end)).  A
// block may decode before its chunk is streamed (it then reads from HBM).
constexpr uint32_t kStreamChunk = 16;
constexpr uint32_t kStreamGroups = 8192;

// Streams the directory entries, slabs and segment areas of blocks [b0, b1]
// of a blob of `bytes` bytes through the caches, eight 16-byte loads in
// flight per lane; the segment byte range comes from the first and last
// directory entries, checked against the layout (a corrupt range is
// skipped).  The loaded words are folded into acc, which the caller keeps
// alive so the loads are not removed.
__device__ __forceinline__ void stream_blocks(const uint8_t* __restrict__ blob, const Layout& L, uint64_t bytes,
                                              uint64_t b0, uint64_t b1, uint32_t& acc)
{
    const uint4* dir = reinterpret_cast<const uint4*>(blob + L.off_dir);
    const uint4* p = reinterpret_cast<const uint4*>(blob);
    const uint64_t d_lo = (L.off_dir + 16 * b0) / 16, dn = b1 + 1 - b0;
    const uint64_t r_lo = (L.off_res + b0 * L.res_stride) / 16, rn = (b1 + 1 - b0) * L.res_stride / 16;
    const uint4 e0 = dir[b0], e1 = dir[b1];
    uint64_t lo = e0.x | ((uint64_t)e0.y << 32);
    uint64_t hi = (e1.x | ((uint64_t)e1.y << 32)) + a16(2ull * e1.z) + a16((uint64_t)((e1.w >> 16) & 0xFF) * e1.z) +
                  a16((uint64_t)(e1.w >> 24) * e1.z) + a16((uint64_t)L.fb * e1.z);
    if (!(lo >= L.off_seg && lo <= hi && hi <= bytes)) lo = hi = L.off_seg;  // corrupt: skip
    const uint64_t s_lo = lo / 16, sn = (hi - lo) / 16;
    const uint64_t tot = dn + rn + sn;  // >= 1
    auto at = [&](uint64_t i) {
        i = i < tot ? i : tot - 1;
        return i < dn ? d_lo + i : i < dn + rn ? r_lo + (i - dn) : s_lo + (i - dn - rn);
    };
    for (uint64_t i0 = threadIdx.x; i0 < tot; i0 += 64 * 8) {
        uint4 v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = p[at(i0 + 64ull * u)];
#pragma unroll
        for (int u = 0; u < 8; u++) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
}

template <int KB, bool RANGE>
__global__ __launch_bounds__(64) void decode_full_kernel(const uint8_t* __restrict__ blob, DecodeArgs a, uint32_t T,
                                                         void* __restrict__ out)
{
    const Layout& L = a.L;
    if (blockIdx.x < T) {
        const uint64_t nch = (a.nblk + kStreamChunk - 1) / kStreamChunk;
        const uint64_t b_end = a.b_first + a.nblk;  // <= L.nblocks
        uint32_t acc = 0;
        for (uint64_t c = blockIdx.x; c < nch; c += T) {
            const uint64_t b0 = a.b_first + c * kStreamChunk;
            const uint64_t b1 = (b0 + kStreamChunk < b_end ? b0 + kStreamChunk : b_end) - 1;
            stream_blocks(blob, L, a.bytes, b0, b1, acc);
        }
        asm volatile("" ::"v"(acc));  // keeps the loads; no instruction is emitted
        return;
    }
    const uint32_t w = blockIdx.x - T;
    const uint64_t rel = (uint64_t)(w % 8) * a.per_xcd + w / 8;
    if (rel >= a.nblk) return;
    decode_block<KB, RANGE>(blob, a, a.b_first + rel, a.raw_cap, out);
}

// Streams the directory entries and segment areas of blocks [b_lo, b_hi]
// through the caches (the approximate decode reads no slab); the segment
// byte range comes from the first and last directory entries, checked
// against the layout.
__global__ __launch_bounds__(256) void touch_blocks_kernel(const uint8_t* __restrict__ blob, Layout L, uint64_t b_lo,
                                                           uint64_t b_hi)
{
    const uint4* dir = reinterpret_cast<const uint4*>(blob + L.off_dir);
    const uint4 d0 = dir[b_lo], d1 = dir[b_hi];
    uint64_t lo = d0.x | ((uint64_t)d0.y << 32);
    uint64_t hi = (d1.x | ((uint64_t)d1.y << 32)) + a16(2ull * d1.z) + a16((uint64_t)((d1.w >> 16) & 0xFF) * d1.z) +
                  a16((uint64_t)(d1.w >> 24) * d1.z) + a16((uint64_t)L.fb * d1.z);
    if (!(lo >= L.off_seg && lo <= hi && hi <= L.blob_bytes)) lo = hi = L.off_seg;
    const uint64_t dlo = (L.off_dir + 16 * b_lo) / 16, dn = b_hi + 1 - b_lo;
    const uint64_t slo = lo / 16, sn = (hi - lo) / 16;
    const uint4* p = reinterpret_cast<const uint4*>(blob);
    uint32_t acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < dn + sn; i += (uint64_t)gridDim.x * 256) {
        const uint4 v = p[i < dn ? dlo + i : slo + (i - dn)];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    asm volatile("" ::"v"(acc));  // keeps the loads; no instruction is emitted
}

// ---------------------------------------------------------------------------
// Point queries
// ---------------------------------------------------------------------------

struct BlockView {
    uint64_t seg_off;
    uint32_t nseg, nkeys, ab, sb;
};

__device__ __forceinline__ BlockView block_view(const uint4& dv)
{
    BlockView v;
    v.seg_off = dv.x | ((uint64_t)dv.y << 32);
    v.nseg = dv.z;
    v.nkeys = (dv.w & 0xFFFF) + 1;
    v.ab = (dv.w >> 16) & 0xFF;
    v.sb = dv.w >> 24;
    return v;
}

// Residual code j of block b, read straight from the blob.
__device__ __forceinline__ uint64_t code_at(const uint8_t* blob, const Layout& L, uint64_t b, uint32_t j)
{
    if (L.w == 0) return 0;
    const uint64_t bitpos = (uint64_t)j * L.w;
    const uint32_t* slab = reinterpret_cast<const uint32_t*>(blob + L.off_res + b * L.res_stride);
    const uint32_t wd = (uint32_t)(bitpos >> 5), sh = (uint32_t)(bitpos & 31);
    uint64_t win = slab[wd];
    if (sh + L.w > 32) win |= (uint64_t)slab[wd + 1] << 32;
    return (win >> sh) & ((1ull << L.w) - 1);
}

// K[i] for i < L.n: directory entry, the segment of position j among the
// block's u16 starts, anchor, slope, one or two slab words.  A directory
// entry inconsistent with the layout (a corrupt blob) gives 0 and sets bad,
// so no read leaves the blob.
template <int KB, bool APPROX = false>
__device__ __forceinline__ uint64_t access_one(const uint8_t* __restrict__ blob, const Layout& L, uint64_t i,
                                               bool& bad)
{
    const uint64_t b = i >> L.log2b;
    const uint32_t j = (uint32_t)(i & ((1ull << L.log2b) - 1));
    const uint4 dv = reinterpret_cast<const uint4*>(blob + L.off_dir)[b];
    if (!dir_ok(dv, L, b, L.blob_bytes)) {
        bad = true;
        return 0;
    }
    const BlockView v = block_view(dv);
    const uint16_t* st = reinterpret_cast<const uint16_t*>(blob + v.seg_off);
    const uint32_t t = find_segment(st, v.nseg, v.nkeys, j);
    const uint8_t* an = blob + v.seg_off + a16(2ull * v.nseg);
    const uint8_t* sl = an + a16((uint64_t)v.ab * v.nseg);
    const uint64_t anchor = load_key<KB>(blob + L.off_first, b) + load_w(an, t, v.ab);
    const uint64_t A = load_w(sl, t, v.sb);
    // the intercept fraction (optimal fit; A d + frac < 2^64 by its cap)
    const uint64_t frac = L.fb ? load_w(sl + a16((uint64_t)v.sb * v.nseg), t, L.fb) : 0;
    const uint64_t pred = anchor + ((A * (uint64_t)(j - st[t]) + frac) >> L.F);
    if constexpr (APPROX) return pred;  // f(i), within eps of K[i]
    return pred + code_at(blob, L, b, j) - L.eps;
}

// First i with K[i] >= x (L.n if none): binary search over first_keys, then
// over the block's segment anchors (segment pruning), then over the decoded
// keys of one segment.  An anchor is its segment's first key, except in
// blobs of the optimal fit (kFlagFrac), whose anchors are intercepts within
// eps of it: there a probe decodes its segment's first key only when x is
// within eps of the intercept.  A directory entry inconsistent with the
// layout, or segment starts out of order, give n and set bad.
template <int KB>
__device__ __forceinline__ uint64_t lower_bound_one(const uint8_t* __restrict__ blob, const Layout& L, uint64_t x,
                                                    bool& bad)
{
    const uint8_t* fk = blob + L.off_first;
    if (L.n == 0 || load_key<KB>(fk, 0) >= x) return 0;
    // last block whose first key is < x
    uint64_t b = 0;
    for (uint64_t step = 1ull << (63 - __clzll((long long)L.nblocks)); step; step >>= 1)
        if (b + step < L.nblocks && load_key<KB>(fk, b + step) < x) b += step;
    const uint4 dv = reinterpret_cast<const uint4*>(blob + L.off_dir)[b];
    if (!dir_ok(dv, L, b, L.blob_bytes)) {
        bad = true;
        return L.n;
    }
    const BlockView v = block_view(dv);
    const uint16_t* st = reinterpret_cast<const uint16_t*>(blob + v.seg_off);
    const uint8_t* an = blob + v.seg_off + a16(2ull * v.nseg);
    const uint8_t* sl = an + a16((uint64_t)v.ab * v.nseg);
    const uint64_t first = load_key<KB>(fk, b);
    const bool free_icpt = (L.flags & kFlagFrac) != 0;
    // first key of segment u: its anchor, or with free intercepts anchor +
    // code - eps (the fraction adds floor(frac / 2^F) = 0 at d = 0)
    auto seg_first = [&](uint32_t u) -> uint64_t {
        uint64_t k = first + load_w(an, u, v.ab);
        if (free_icpt) {
            k += code_at(blob, L, b, st[u]) - L.eps;
            if constexpr (KB == 4) k &= 0xFFFFFFFFull;
        }
        return k;
    };
    // last segment whose first key is < x (binary search: on heavy-tailed
    // key distributions the anchors of sparse blocks are too uneven for a
    // proportional guess to pay off)
    uint32_t t = 0;
    uint64_t Kt = first;  // first key of segment t (segment 0 starts the block)
    // With free intercepts, the stored delta = intercept - first is within eps
    // of K[start] - first, and exact (no wrap modulo 2^64) for 4-byte keys or
    // when first >= eps; then a probe decides from the delta alone unless it
    // lies within eps of x - first, and only the segment found is decoded.
    const bool by_delta = free_icpt && (KB == 4 || first >= L.eps);
    if (by_delta) {
        const uint64_t X = x - first;  // >= 1; X + eps does not overflow (first >= eps)
        for (uint32_t step = pow2_floor(v.nseg); step; step >>= 1) {
            if (t + step < v.nseg) {
                const uint64_t dlt = load_w(an, t + step, v.ab);
                const bool below = (X > L.eps && dlt < X - L.eps) ? true
                                   : dlt >= X + L.eps            ? false
                                                                 : seg_first(t + step) < x;
                if (below) t += step;
            }
        }
        if (t != 0) Kt = seg_first(t);
    } else {
        for (uint32_t step = pow2_floor(v.nseg); step; step >>= 1) {
            if (t + step < v.nseg) {
                const uint64_t k = seg_first(t + step);
                if (k < x) {
                    t += step;
                    Kt = k;
                }
            }
        }
    }
    const uint32_t s = st[t];
    const uint32_t e = t + 1 < v.nseg ? st[t + 1] : v.nkeys;
    if (!(s < e && e <= v.nkeys)) {  // corrupt starts: the window below would leave the slab
        bad = true;
        return L.n;
    }
    const uint64_t anchor = first + load_w(an, t, v.ab);
    const uint64_t A = load_w(sl, t, v.sb);
    const uint64_t frac = L.fb ? load_w(sl + a16((uint64_t)v.sb * v.nseg), t, L.fb) : 0;
    // The eps window, from the model alone (no memory reads): with
    // G(d) = floor((A d + frac) / 2^F) and dl = intercept - K[s] (0 when
    // anchored; |dl| <= eps, exact as a signed difference modulo 2^64), key
    // s + d is certainly below x when G(d) + dl + eps < x - K[s], and
    // certainly not when G(d) + dl - eps >= x - K[s]; G is non-decreasing in
    // d.  Sums that would pass 2^64 certify nothing.
    const uint64_t X = x - Kt;                              // >= 1
    const int64_t dl = (int64_t)(anchor - Kt);
    const uint64_t up = (uint64_t)(dl + (int64_t)L.eps);    // in [0, 2 eps]
    const uint64_t down = (uint64_t)((int64_t)L.eps - dl);  // in [0, 2 eps]
    const bool down_ok = X <= ~0ull - down;
    auto G = [&](uint32_t d) -> uint64_t { return (A * (uint64_t)d + frac) >> L.F; };
    auto below = [&](uint32_t d) -> bool {
        const uint64_t g = G(d);
        return g <= ~0ull - up && g + up < X;
    };
    auto above = [&](uint32_t d) -> bool { return down_ok && G(d) >= X + down; };
    const uint32_t len = e - s;
    uint32_t da = 1, db = len;  // first d in [1, len) not certainly below x, else len
    while (da < db) {
        const uint32_t m = (da + db) >> 1;
        if (below(m)) da = m + 1;
        else db = m;
    }
    uint32_t dc = da, dd = len;  // first d in [da, len) certainly not below x, else len
    while (dc < dd) {
        const uint32_t m = (dc + dd) >> 1;
        if (above(m)) dd = m;
        else dc = m + 1;
    }
    // keys in the window: first one >= x, else s + dc (which is e or a key >= x)
    uint32_t lo = s + da, hi = s + dc;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        uint64_t k = anchor + ((A * (uint64_t)(mid - s) + frac) >> L.F) + code_at(blob, L, b, mid) - L.eps;
        if constexpr (KB == 4) k &= 0xFFFFFFFFull;
        if (k >= x) hi = mid;
        else lo = mid + 1;
    }
    return (b << L.log2b) + lo;
}

template <int KB>
__global__ __launch_bounds__(256) void access_kernel(const uint8_t* __restrict__ blob, Layout L,
                                                     const uint64_t* __restrict__ idx, uint64_t m,
                                                     void* __restrict__ out, uint32_t* __restrict__ flags)
{
    bool bad = false, corrupt = false;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m; q += stride) {
        const uint64_t i = idx[q];
        if (i >= L.n) {
            store_key<KB>(out, q, 0);
            bad = true;
            continue;
        }
        store_key<KB>(out, q, access_one<KB>(blob, L, i, corrupt));
    }
    if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(flags, kFlagRange);
    if (__ballot(corrupt) != 0 && lane_id() == 0) atomicOr(flags, kFlagBadList);
}

template <int KB>
__global__ __launch_bounds__(256) void lower_bound_kernel(const uint8_t* __restrict__ blob, Layout L,
                                                          const void* __restrict__ qs, uint64_t m,
                                                          uint64_t* __restrict__ pos)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    bool corrupt = false;  // n answers for queries in an inconsistent block; there is no flag word
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m; q += stride)
        pos[q] = lower_bound_one<KB>(blob, L, load_key<KB>(qs, q), corrupt);
}

// ---------------------------------------------------------------------------
// Quantiles and list AND / OR (Sec. III-C, III-A)
// ---------------------------------------------------------------------------

// out[i] = K[min(floor(n k_i / q), n - 1)]; APPROX: f of that index.
template <int KB, bool APPROX>
__global__ __launch_bounds__(256) void quantile_kernel(const uint8_t* __restrict__ blob, Layout L,
                                                       const uint64_t* __restrict__ ks, uint64_t q, uint64_t m,
                                                       void* __restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += stride) {
        const unsigned __int128 prod = (unsigned __int128)L.n * ks[t];
        const unsigned __int128 i = prod / q;
        const uint64_t idx = i < (unsigned __int128)(L.n - 1) ? (uint64_t)i : L.n - 1;
        bool corrupt = false;  // 0 for an index in an inconsistent block; there is no flag word
        store_key<KB>(out, t, access_one<KB, APPROX>(blob, L, idx, corrupt));
    }
}

constexpr uint32_t kSetTile = 1024;  // elements per tile of the set operations (one per thread)
static_assert(kSetTile == kSetTileKeys, "host workspace plan uses the same tile");

// x is a key of the compressed list (segment-pruned lower_bound, then one access)
template <int KB>
__device__ __forceinline__ bool contains_one(const uint8_t* __restrict__ blob, const Layout& L, uint64_t x)
{
    bool corrupt = false;
    const uint64_t p = lower_bound_one<KB>(blob, L, x, corrupt);
    if (p >= L.n || corrupt) return false;
    uint64_t v = access_one<KB>(blob, L, p, corrupt);
    if constexpr (KB == 4) v &= 0xFFFFFFFFull;
    return v == x && !corrupt;
}

// first index i of the decoded sorted array with a[i] >= x
template <int KB>
__device__ __forceinline__ uint64_t lb_sorted(const void* __restrict__ a, uint64_t n, uint64_t x)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (load_key<KB>(a, mid) < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void tile_count(uint32_t f, uint64_t* __restrict__ cnt, uint64_t tile)
{
    uint64_t tot;
    block_excl_sum<kSetTile>(f, &tot);
    if (threadIdx.x == 0) cnt[tile] = tot;
}

// AND, probing the compressed list B with the decoded keys of A: flag[i] =
// A[i] is the first copy of its value and B holds it.  B is never decoded;
// each probe reads one block's directory entry, the anchors of that block
// and one segment -- the segment pruning of Sec. III-A.
template <int KB>
__global__ __launch_bounds__(kSetTile) void and_flags_kernel(const uint8_t* __restrict__ blob_b, Layout Lb,
                                                             const void* __restrict__ a, uint64_t na,
                                                             uint8_t* __restrict__ flags, uint64_t* __restrict__ cnt,
                                                             uint64_t tile0)
{
    const uint64_t tile = tile0 + blockIdx.x;
    const uint64_t i = tile * kSetTile + threadIdx.x;
    uint32_t f = 0;
    if (i < na) {
        const uint64_t x = load_key<KB>(a, i);
        f = (i == 0 || load_key<KB>(a, i - 1) != x) && contains_one<KB>(blob_b, Lb, x);
        flags[i] = (uint8_t)f;
    }
    tile_count(f, cnt, tile);
}

// OR flags over the decoded lists: tiles [0, ta) cover A, the rest B.
// fa[i] = A[i] is the first copy of its value; fb[j] = B[j] is the first
// copy of its value and A does not hold it.
template <int KB>
__global__ __launch_bounds__(kSetTile) void or_flags_kernel(const void* __restrict__ a, uint64_t na,
                                                            const void* __restrict__ b, uint64_t nb, uint64_t ta,
                                                            uint8_t* __restrict__ fa, uint8_t* __restrict__ fb,
                                                            uint64_t* __restrict__ cnt, uint64_t tile0)
{
    const uint64_t tile = tile0 + blockIdx.x;
    uint32_t f = 0;
    if (tile < ta) {
        const uint64_t i = tile * kSetTile + threadIdx.x;
        if (i < na) {
            const uint64_t x = load_key<KB>(a, i);
            f = i == 0 || load_key<KB>(a, i - 1) != x;
            fa[i] = (uint8_t)f;
        }
    } else {
        const uint64_t j = (tile - ta) * kSetTile + threadIdx.x;
        if (j < nb) {
            const uint64_t x = load_key<KB>(b, j);
            const uint64_t p = lb_sorted<KB>(a, na, x);
            f = (j == 0 || load_key<KB>(b, j - 1) != x) && !(p < na && load_key<KB>(a, p) == x);
            fb[j] = (uint8_t)f;
        }
    }
    tile_count(f, cnt, tile);
}

// One workgroup: exclusive scans of the tile counts of [0, ta) and of
// [ta, ta + tb) in place; totals to tot[0], tot[1]; count = tot[0] + tot[1].
__global__ __launch_bounds__(1024) void set_tiles_scan_kernel(uint64_t* __restrict__ cnt, uint64_t ta, uint64_t tb,
                                                              uint64_t* __restrict__ tot, uint64_t* __restrict__ count)
{
    uint64_t sums[2] = {0, 0};
    for (int part = 0; part < 2; part++) {
        uint64_t* c = cnt + (part ? ta : 0);
        const uint64_t nt = part ? tb : ta;
        uint64_t carry = 0;
        for (uint64_t t0 = 0; t0 < nt; t0 += 1024) {
            const uint64_t t = t0 + threadIdx.x;
            const uint64_t v = t < nt ? c[t] : 0;
            uint64_t all;
            const uint64_t ex = block_excl_sum<1024>(v, &all);
            if (t < nt) c[t] = carry + ex;
            carry += all;
        }
        sums[part] = carry;
    }
    if (threadIdx.x == 0) {
        tot[0] = sums[0];
        tot[1] = sums[1];
        *count = sums[0] + sums[1];
    }
}

// AND output: the flagged keys of A at their exclusive prefix positions.
template <int KB>
__global__ __launch_bounds__(kSetTile) void and_scatter_kernel(const void* __restrict__ a, uint64_t na,
                                                               const uint8_t* __restrict__ flags,
                                                               const uint64_t* __restrict__ off, void* __restrict__ out,
                                                               uint64_t tile0)
{
    const uint64_t tile = tile0 + blockIdx.x;
    const uint64_t i = tile * kSetTile + threadIdx.x;
    const uint32_t f = i < na ? flags[i] : 0u;
    uint64_t tot;
    const uint64_t ex = block_excl_sum<kSetTile>(f, &tot);
    if (f) store_key<KB>(out, off[tile] + ex, load_key<KB>(a, i));
}

// OR ranks: P[i] = flags before i (exclusive prefix), P[n] = total.
// (launched over ceil((n + 1) / kSetTile) tiles, so that index n is covered)
__global__ __launch_bounds__(kSetTile) void prefix_kernel(const uint8_t* __restrict__ flags, uint64_t n,
                                                          const uint64_t* __restrict__ off,
                                                          const uint64_t* __restrict__ total,
                                                          uint64_t* __restrict__ P, uint64_t tile0)
{
    const uint64_t tile = tile0 + blockIdx.x;
    const uint64_t i = tile * kSetTile + threadIdx.x;
    const uint32_t f = i < n ? flags[i] : 0u;
    uint64_t tot;
    const uint64_t ex = block_excl_sum<kSetTile>(f, &tot);
    if (i < n) P[i] = off[tile] + ex;
    if (i == n) P[n] = *total;
}

// OR output: a kept key x of A goes to (distinct A before it) + (B-only keys
// < x); a kept key of B to (distinct A < x) + (B-only keys before it): its
// rank among the distinct keys of A u B.
template <int KB>
__global__ __launch_bounds__(kSetTile) void or_scatter_kernel(const void* __restrict__ a, uint64_t na,
                                                              const void* __restrict__ b, uint64_t nb, uint64_t ta,
                                                              const uint8_t* __restrict__ fa,
                                                              const uint8_t* __restrict__ fb,
                                                              const uint64_t* __restrict__ PA,
                                                              const uint64_t* __restrict__ PB, void* __restrict__ out,
                                                              uint64_t tile0)
{
    const uint64_t tile = tile0 + blockIdx.x;
    if (tile < ta) {
        const uint64_t i = tile * kSetTile + threadIdx.x;
        if (i < na && fa[i]) {
            const uint64_t x = load_key<KB>(a, i);
            store_key<KB>(out, PA[i] + PB[lb_sorted<KB>(b, nb, x)], x);
        }
    } else {
        const uint64_t j = (tile - ta) * kSetTile + threadIdx.x;
        if (j < nb && fb[j]) {
            const uint64_t x = load_key<KB>(b, j);
            store_key<KB>(out, PB[j] + PA[lb_sorted<KB>(a, na, x)], x);
        }
    }
}

// ---------------------------------------------------------------------------
// Request batches (the server's launches)
// ---------------------------------------------------------------------------

// One launch serves a batch of requests: waves [0, range_items) decode one
// block of one range request each (requests found by binary search over
// item_off), the remaining waves answer 64 point requests each.  Outputs go
// to the server's arena at each request's offset.
template <int KB>
__global__ __launch_bounds__(64) void serve_kernel(const uint8_t* __restrict__ blob, ServeArgs s,
                                                   const ServeRange* __restrict__ ranges,
                                                   const ServePoint* __restrict__ points, uint8_t* __restrict__ arena)
{
    const uint64_t w = blockIdx.x;
    if (w < s.range_items) {
        uint32_t lo = 0, hi = s.nrange;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (ranges[mid].item_off <= w) lo = mid;
            else hi = mid;
        }
        const ServeRange R = ranges[lo];
        DecodeArgs d{};
        d.L = s.L;
        d.begin = R.a;
        d.end = R.b;
        d.raw_cap = s.raw_cap;
        d.bytes = s.L.blob_bytes;
        d.flags = nullptr;
        decode_block<KB, true>(blob, d, (R.a >> s.L.log2b) + (w - R.item_off), s.raw_cap, arena + R.out_off);
        return;
    }
    const uint64_t q = (w - s.range_items) * 64 + threadIdx.x;
    if (q >= s.npoint) return;
    const ServePoint P = points[q];
    bool corrupt = false;  // the server's blob passed lc_info; an inconsistent block answers 0 / n
    if (P.op == kServeAccess) store_key<KB>(arena + P.out_off, 0, access_one<KB>(blob, s.L, P.key, corrupt));
    else *reinterpret_cast<uint64_t*>(arena + P.out_off) = lower_bound_one<KB>(blob, s.L, P.key, corrupt);
}

// ---------------------------------------------------------------------------
// Batches of lists
// ---------------------------------------------------------------------------

constexpr uint32_t kMaxCands = 8;

// Candidate error bounds of a size pass (kernel argument).
struct Cands {
    uint32_t eps[kMaxCands];
    uint32_t n;
};

// Blob v1 layout of a list of n keys at eps (mirrors the host's layout).
__device__ __forceinline__ Layout list_layout(const BatchArgs& a, uint64_t n, uint32_t eps)
{
    Layout L;
    const uint64_t B = 1ull << a.log2b;
    L.n = n;
    L.nblocks = (n + B - 1) >> a.log2b;
    L.kb = a.kb;
    L.log2b = a.log2b;
    L.F = a.F;
    L.eps = eps;
    L.w = eps ? 64 - __clzll((long long)(2ull * eps)) : 0u;  // smallest w with 2^w > 2 eps
    L.res_stride = a16((B * L.w + 7) / 8);
    L.off_first = kHeaderBytes;
    L.off_dir = L.off_first + a16(L.nblocks * a.kb);
    L.off_res = L.off_dir + 16 * L.nblocks;
    L.off_seg = L.off_res + L.nblocks * L.res_stride;
    L.max_nseg = 0;
    L.max_seg_bytes = 0;
    L.blob_bytes = 0;
    L.flags = a.fit == LC_FIT_OPT ? kFlagFrac : 0u;  // the optimal fit stores intercept fractions
    L.fb = L.flags ? frac_bytes(a.F) : 0u;
    return L;
}

// Does list li fit the buffers of the batch?  Keys (or outputs) [key_off,
// key_off + n) inside the a.nkeys given, its blocks and 4-block groups inside
// the plan's totals, eps <= max_eps and, when the blob is used, a 16-byte
// aligned slot inside the buffer that holds the list's worst-case blob.
__device__ __forceinline__ bool list_fits(const lc_batch_list& li, const BatchArgs& a, const Layout& L,
                                          uint32_t eps, bool use_blob)
{
    const uint64_t B = 1ull << a.log2b;
    bool ok = li.n <= a.nkeys && li.key_off <= a.nkeys - li.n && eps <= a.max_eps && li.n <= (1ull << 40);
    ok = ok && li.block_off <= a.total_blocks && L.nblocks <= a.total_blocks - li.block_off;
    ok = ok && li.group_off <= a.total_groups && (L.nblocks + 3) / 4 <= a.total_groups - li.group_off;
    if (use_blob) {
        const uint64_t worst = L.off_seg + L.nblocks * (a16(2 * B) + 2 * a16(8 * B) + a16(L.fb * B));
        ok = ok && (li.blob_off & 15) == 0 && li.blob_off <= a.blob_cap && li.blob_cap <= a.blob_cap - li.blob_off &&
             worst <= li.blob_cap;
    }
    return ok;
}

// The list owning item x: the last l with off(l) <= x.  Offsets are
// non-decreasing in a planned table (empty lists repeat their successor's).
template <bool BY_GROUP>
__device__ __forceinline__ uint32_t find_list(const lc_batch_list* __restrict__ lists, uint32_t nlists, uint64_t x)
{
    uint32_t lo = 0, hi = nlists;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        const uint64_t off = BY_GROUP ? lists[mid].group_off : lists[mid].block_off;
        if (off <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// find_list for a whole wave with x uniform: each round the 64 lanes probe
// 64 evenly spaced lists of the remaining range at once and the ballot of
// "offset <= x" narrows it to one stride, so 4096 lists take two rounds of
// loads instead of twelve dependent ones.
template <bool BY_GROUP>
__device__ __forceinline__ uint32_t find_list_wave(const lc_batch_list* __restrict__ lists, uint32_t nlists,
                                                   uint64_t x)
{
    const uint32_t lane = lane_id();
    uint32_t lo = 0, n = nlists;
    while (n > 1) {
        const uint32_t step = (n + 63) / 64;
        const uint32_t idx = lo + lane * step;
        const bool ok = lane == 0 || (idx < lo + n && (BY_GROUP ? lists[idx].group_off : lists[idx].block_off) <= x);
        const uint64_t mask = __ballot(ok);
        const uint32_t k = 63 - __clzll(mask);
        lo += k * step;
        n = n - k * step < step ? n - k * step : step;
    }
    return lo;
}

// Workspace of one list: block infos and segment records at its block offset.
__device__ __forceinline__ Workspace list_ws(const Workspace& ws, uint64_t block_off, uint32_t log2b, uint64_t blk_off)
{
    Workspace w;
    w.blk = ws.blk + blk_off;
    w.tiles = nullptr;
    const uint64_t rec = block_off << log2b;
    w.seg_start = ws.seg_start ? ws.seg_start + rec : nullptr;
    w.seg_delta = ws.seg_delta ? ws.seg_delta + rec : nullptr;
    w.seg_A = ws.seg_A ? ws.seg_A + rec : nullptr;
    w.seg_frac = ws.seg_frac ? ws.seg_frac + rec : nullptr;
    return w;
}

// Fit over every (list, 4-block group) work item of the batch, one wave per
// item.  SIZES: the size pass, once per candidate eps (item index
// c * total_groups + g), block infos only.
template <int KB, bool SIZES>
__global__ __launch_bounds__(64) void batch_fit_kernel(const void* __restrict__ keys,
                                                       const lc_batch_list* __restrict__ lists, BatchArgs a,
                                                       Cands cands, uint8_t* __restrict__ blob, Workspace ws,
                                                       uint32_t* __restrict__ stats, uint64_t item0)
{
    const uint64_t item = item0 + blockIdx.x;
    const uint64_t cand = SIZES ? item / a.total_groups : 0;
    const uint64_t g = SIZES ? item % a.total_groups : item;
    const uint32_t l = find_list_wave<true>(lists, a.nlists, g);
    const lc_batch_list li = lists[l];
    const uint32_t eps = SIZES ? cands.eps[cand] : li.eps;
    const Layout L = list_layout(a, li.n, eps);
    const uint64_t local = g - li.group_off;
    if (!list_fits(li, a, L, eps, !SIZES) || local >= (L.nblocks + 3) / 4) {
        if (threadIdx.x == 0) atomicOr(stats, kFlagBadList);
        return;
    }
    const Workspace w = list_ws(ws, li.block_off, a.log2b, cand * a.total_blocks + li.block_off);
    const uint8_t* k = reinterpret_cast<const uint8_t*>(keys) + li.key_off * KB;
    fit_rows<KB, SIZES>(k, L, SIZES ? nullptr : blob + li.blob_off, w, stats, local * 4);
}

// The fewest-segment (FIT = LC_FIT_MIN) or optimal (LC_FIT_OPT) fit over the
// blocks of a batch, one workgroup per block as the single-list kernels:
// item = a batch block, or (candidate, block) for the size pass (SIZES:
// block infos only).  The block's list is found and checked like
// batch_fit_kernel's.
template <int KB, bool SIZES, uint32_t FIT>
__global__ __launch_bounds__(64) void batch_block_fit_kernel(const void* __restrict__ keys,
                                                             const lc_batch_list* __restrict__ lists, BatchArgs a,
                                                             Cands cands, uint8_t* __restrict__ blob, Workspace ws,
                                                             uint32_t* __restrict__ stats, uint64_t item0)
{
    const uint64_t item = item0 + blockIdx.x;
    const uint64_t cand = SIZES ? item / a.total_blocks : 0;
    const uint64_t gb = SIZES ? item % a.total_blocks : item;
    const lc_batch_list li = lists[find_list_wave<false>(lists, a.nlists, gb)];
    const uint32_t eps = SIZES ? cands.eps[cand] : li.eps;
    const Layout L = list_layout(a, li.n, eps);
    const uint64_t b = gb - li.block_off;
    if (!list_fits(li, a, L, eps, !SIZES) || gb < li.block_off || b >= L.nblocks) {
        if (threadIdx.x == 0) atomicOr(stats, kFlagBadList);
        return;
    }
    const Workspace w = list_ws(ws, li.block_off, a.log2b, cand * a.total_blocks + li.block_off);
    const uint8_t* k = reinterpret_cast<const uint8_t*>(keys) + li.key_off * KB;
    uint8_t* bl = SIZES ? nullptr : blob + li.blob_off;
    if (FIT == LC_FIT_MIN)
        fit_min_block<KB, SIZES>(k, L, bl, w, stats, b);
    else
        fit_opt_block<KB, SIZES>(k, L, bl, w, stats, b);
}

// Lane-per-block fit over the blocks of a batch (lanes_fit): item = a
// 64-block group of the batch, or (candidate, group) for the size pass
// (SIZES: block infos only).  Each lane finds its block's list by binary
// search over the block offsets and checks it like batch_fit_kernel.
template <int KB, bool SIZES>
__global__ __launch_bounds__(64) void batch_lanes_kernel(const void* __restrict__ keys,
                                                         const lc_batch_list* __restrict__ lists, BatchArgs a,
                                                         Cands cands, uint8_t* __restrict__ blob, Workspace ws,
                                                         uint32_t* __restrict__ stats, uint64_t item0)
{
    const uint64_t item = item0 + blockIdx.x;
    const uint64_t groups = (a.total_blocks + 63) / 64;
    const uint64_t cand = SIZES ? item / groups : 0;
    const uint64_t gb = (SIZES ? item % groups : item) * 64 + threadIdx.x;
    const uint32_t B = 1u << a.log2b;
    LaneBlock in;
    in.koff = 0;
    in.nb = 0;
    in.has_prev = false;
    in.eps = 0;
    in.st = nullptr;
    in.dl = nullptr;
    in.sa = nullptr;
    in.info = nullptr;
    in.first_dst = nullptr;
    bool bad = false;
    if (gb < a.total_blocks) {
        const uint32_t l = find_list<false>(lists, a.nlists, gb);
        const lc_batch_list li = lists[l];
        const uint32_t eps = SIZES ? cands.eps[cand] : li.eps;
        const Layout L = list_layout(a, li.n, eps);
        const uint64_t lb = gb - li.block_off;
        if (!list_fits(li, a, L, eps, !SIZES) || lb >= L.nblocks) {
            bad = true;
        } else {
            const Workspace w = list_ws(ws, li.block_off, a.log2b, cand * a.total_blocks + li.block_off);
            const uint64_t rec = lb << a.log2b;
            in.nb = (li.n - rec) < B ? (uint32_t)(li.n - rec) : B;
            in.koff = li.key_off + rec;
            in.has_prev = lb > 0;
            in.eps = eps;
            if (!SIZES) {
                in.st = w.seg_start + rec;
                in.dl = w.seg_delta + rec;
                in.sa = w.seg_A + rec;
                in.first_dst = blob + li.blob_off + L.off_first + lb * KB;
            }
            in.info = w.blk + lb;
        }
    }
    if (__ballot(bad) != 0 && threadIdx.x == 0) atomicOr(stats, kFlagBadList);
    lanes_fit<KB, !SIZES>(in, keys, a.nkeys, a.log2b, a.F, stats);
}

// Residual codes of every block of a batch after batch_lanes_kernel, one
// wave per block (code_pack_block on the list's slot).
template <int KB>
__global__ __launch_bounds__(64) void batch_code_pack_kernel(const void* __restrict__ keys,
                                                             const lc_batch_list* __restrict__ lists, BatchArgs a,
                                                             uint8_t* __restrict__ blob, Workspace ws, uint64_t b0)
{
    const uint64_t gb = b0 + blockIdx.x;  // the launcher keeps gb < total_blocks
    const uint32_t l = find_list_wave<false>(lists, a.nlists, gb);
    const lc_batch_list li = lists[l];
    const Layout L = list_layout(a, li.n, li.eps);
    const uint64_t lb = gb - li.block_off;
    if (!list_fits(li, a, L, li.eps, true) || lb >= L.nblocks) return;  // flagged by the fit
    const Workspace w = list_ws(ws, li.block_off, a.log2b, li.block_off);
    const uint64_t rec = lb << a.log2b;
    code_pack_block<KB>(reinterpret_cast<const uint8_t*>(keys) + (li.key_off + rec) * KB, w.blk[lb],
                        w.seg_start + rec, w.seg_delta + rec, w.seg_A + rec, a.log2b, L.res_stride, L.w, li.eps,
                        a.F, blob + li.blob_off + L.off_res + lb * L.res_stride);
}

template <int NT>
__device__ __forceinline__ uint64_t block_max(uint64_t v)
{
    __shared__ uint64_t s_m[NT / 64];
    v = wave_max(v);
    if (lane_id() == 0) s_m[threadIdx.x / 64] = v;
    __syncthreads();
    uint64_t m = 0;
    for (uint32_t k = 0; k < NT / 64; k++) m = s_m[k] > m ? s_m[k] : m;
    __syncthreads();
    return m;
}

// One workgroup per list (per candidate and list for the size pass): scan
// of the blocks' segment-area bytes, then (unless SIZES) the directory, the
// header and the first-key padding of the list's blob.  sizes[c * nlists + l]
// receives the blob size (~0 for a list that does not fit the buffers).
template <bool SIZES>
__global__ __launch_bounds__(256) void batch_scan_kernel(const lc_batch_list* __restrict__ lists, BatchArgs a,
                                                         Cands cands, uint8_t* __restrict__ blob, Workspace ws,
                                                         uint64_t* __restrict__ sizes, uint32_t* __restrict__ stats,
                                                         uint64_t item0)
{
    const uint64_t item = item0 + blockIdx.x;
    const uint32_t l = (uint32_t)(item % a.nlists);
    const uint64_t cand = item / a.nlists;
    const lc_batch_list li = lists[l];
    const uint32_t eps = SIZES ? cands.eps[cand] : li.eps;
    const Layout L = list_layout(a, li.n, eps);
    if (!list_fits(li, a, L, eps, !SIZES)) {
        if (threadIdx.x == 0) {
            atomicOr(stats, kFlagBadList);
            if (sizes) sizes[item] = ~0ull;
        }
        return;
    }
    const BlockInfo* blk = ws.blk + cand * a.total_blocks + li.block_off;
    uint8_t* out = SIZES ? nullptr : blob + li.blob_off;
    uint64_t carry = 0, nseg_total = 0, max_nseg = 0, max_area = 0;
    for (uint64_t b0 = 0; b0 < L.nblocks; b0 += 256) {
        const uint64_t b = b0 + threadIdx.x;
        BlockInfo bi = {};
        bool bad = false;
        if (b < L.nblocks) {
            bi = blk[b];
            // block infos of a planned table were all written by the fit
            const uint64_t left = L.n - (b << L.log2b);
            const uint32_t want = left < (1ull << L.log2b) ? (uint32_t)left : (1u << L.log2b);
            const uint32_t ab = bi.ab, sb = bi.sb;
            bad = bi.nkeys != want || bi.nseg < 1 || bi.nseg > want || !ab || !sb || ab > 8 || sb > 8 ||
                  (ab & (ab - 1)) || (sb & (sb - 1)) ||
                  bi.seg_bytes != a16(2ull * bi.nseg) + a16((uint64_t)ab * bi.nseg) + a16((uint64_t)sb * bi.nseg) +
                                      a16((uint64_t)L.fb * bi.nseg);
            if (bad) bi = BlockInfo{};
        }
        if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(stats, kFlagBadList);
        uint64_t tot, tot_n;
        const uint64_t ex = block_excl_sum<256>(bi.seg_bytes, &tot);
        block_excl_sum<256>(bi.nseg, &tot_n);
        if (!SIZES && b < L.nblocks) {
            const uint64_t seg_off = L.off_seg + carry + ex;
            const uint32_t w3 = (bi.nkeys - 1) | ((uint32_t)bi.ab << 16) | ((uint32_t)bi.sb << 24);
            reinterpret_cast<uint4*>(out + L.off_dir)[b] = make_uint4((uint32_t)seg_off, (uint32_t)(seg_off >> 32),
                                                                      bi.nseg, w3);
        }
        carry += tot;
        nseg_total += tot_n;
        max_nseg = b < L.nblocks && bi.nseg > max_nseg ? bi.nseg : max_nseg;
        max_area = b < L.nblocks && bi.seg_bytes > max_area ? bi.seg_bytes : max_area;
    }
    max_nseg = block_max<256>(max_nseg);
    max_area = block_max<256>(max_area);
    const uint64_t blob_bytes = L.off_seg + carry;
    if (threadIdx.x == 0) {
        if (sizes) sizes[item] = blob_bytes;
        if (!SIZES) {
            write_header(out, L, nseg_total, max_nseg, max_area, blob_bytes);
            atomicMax(stats + 1, (uint32_t)max_area);
        }
    }
    if (!SIZES) {
        const uint64_t fk_end = L.off_first + L.nblocks * L.kb;
        if (threadIdx.x < L.off_dir - fk_end) out[fk_end + threadIdx.x] = 0;
    }
}

// Segment areas of every block of the batch: kEmitLanes lanes per block.
__global__ __launch_bounds__(256) void batch_emit_kernel(const lc_batch_list* __restrict__ lists, BatchArgs a,
                                                         uint8_t* __restrict__ blob, Workspace ws, uint64_t blk0)
{
    const uint64_t gb = blk0 + (uint64_t)blockIdx.x * (256 / kEmitLanes) + threadIdx.x / kEmitLanes;
    if (gb >= a.total_blocks) return;
    const uint32_t l = find_list<false>(lists, a.nlists, gb);
    const lc_batch_list li = lists[l];
    const Layout L = list_layout(a, li.n, li.eps);
    const uint64_t b = gb - li.block_off;
    if (!list_fits(li, a, L, li.eps, true) || b >= L.nblocks) return;  // flagged by the fit
    const uint4 dv = reinterpret_cast<const uint4*>(blob + li.blob_off + L.off_dir)[b];
    if (!dir_ok(dv, L, b, li.blob_cap)) return;  // flagged by the scan
    emit_block<kEmitLanes>(list_ws(ws, li.block_off, a.log2b, li.block_off), L, blob + li.blob_off, b);
}

// Decode of every block of the batch, one wave per block, XCD-major as the
// single-list decode.  List l's keys go to out + key_off * KB.
template <int KB>
__device__ __forceinline__ bool batch_block(const lc_batch_list* __restrict__ lists, const BatchArgs& a, uint64_t gb,
                                            lc_batch_list* li, Layout* L, uint64_t* b)
{
    const uint32_t l = find_list_wave<false>(lists, a.nlists, gb);
    *li = lists[l];
    *L = list_layout(a, li->n, li->eps);
    *b = gb - li->block_off;
    return list_fits(*li, a, *L, li->eps, true) && *b < L->nblocks;
}

template <int KB>
__global__ __launch_bounds__(64) void batch_decode_kernel(const uint8_t* __restrict__ blob,
                                                          const lc_batch_list* __restrict__ lists, BatchArgs a,
                                                          uint64_t blk0, uint64_t nblk, uint64_t per_xcd,
                                                          uint32_t raw_cap, void* __restrict__ out,
                                                          uint32_t* __restrict__ stats)
{
    const uint64_t rel = (uint64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (rel >= nblk) return;
    lc_batch_list li;
    DecodeArgs d{};
    uint64_t b;
    if (!batch_block<KB>(lists, a, blk0 + rel, &li, &d.L, &b)) {
        if (threadIdx.x == 0) atomicOr(stats, kFlagBadList);
        return;
    }
    d.begin = 0;
    d.end = li.n;
    d.raw_cap = raw_cap;
    d.bytes = li.blob_cap;
    d.flags = stats;
    // a whole list: no range checks per key (the block's own key count ends it)
    decode_block<KB, false>(blob + li.blob_off, d, b, raw_cap, reinterpret_cast<uint8_t*>(out) + li.key_off * KB);
}

// ---- AND over pairs of lists of a batch ------------------------------------

// The pair owning item x (a probe block or key): the last p with off(p) <= x.
template <bool BY_BLOCK>
__device__ __forceinline__ uint32_t find_pair(const lc_list_pair* __restrict__ pairs, uint32_t npairs, uint64_t x)
{
    uint32_t lo = 0, hi = npairs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((BY_BLOCK ? pairs[mid].block_off : pairs[mid].key_off) <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Does the pair fit the buffers?  Both lists inside the batch, their slots
// inside the blob buffer, the probe keys and blocks inside the plan's totals.
__device__ __forceinline__ bool pair_fits(const lc_list_pair& pr, const lc_batch_list* __restrict__ lists,
                                          const BatchArgs& a, uint64_t total_keys, uint64_t total_blocks,
                                          lc_batch_list* lp, lc_batch_list* lt, Layout* Lp, Layout* Lt)
{
    if (pr.probe >= a.nlists || pr.target >= a.nlists) return false;
    *lp = lists[pr.probe];
    *lt = lists[pr.target];
    *Lp = list_layout(a, lp->n, lp->eps);
    *Lt = list_layout(a, lt->n, lt->eps);
    Lp->blob_bytes = lp->blob_cap;  // point queries check directory entries against the slot
    Lt->blob_bytes = lt->blob_cap;
    return list_fits(*lp, a, *Lp, lp->eps, true) && list_fits(*lt, a, *Lt, lt->eps, true) && pr.n == lp->n &&
           pr.key_off <= total_keys && pr.n <= total_keys - pr.key_off && pr.block_off <= total_blocks &&
           Lp->nblocks <= total_blocks - pr.block_off;
}

// Probe lists of all pairs decoded into the workspace: one wave per block.
template <int KB>
__global__ __launch_bounds__(64) void pair_decode_kernel(const uint8_t* __restrict__ blob,
                                                         const lc_batch_list* __restrict__ lists, BatchArgs a,
                                                         const lc_list_pair* __restrict__ pairs, uint32_t npairs,
                                                         uint64_t total_keys, uint64_t total_blocks, uint64_t blk0,
                                                         uint64_t nblk, uint64_t per_xcd, uint32_t raw_cap,
                                                         void* __restrict__ keys, uint32_t* __restrict__ stats)
{
    const uint64_t rel = (uint64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (rel >= nblk) return;
    const uint64_t gb = blk0 + rel;
    const lc_list_pair pr = pairs[find_pair<true>(pairs, npairs, gb)];
    lc_batch_list lp, lt;
    DecodeArgs d{};
    Layout Lt;
    if (!pair_fits(pr, lists, a, total_keys, total_blocks, &lp, &lt, &d.L, &Lt)) {
        if (threadIdx.x == 0) atomicOr(stats, kFlagBadList);
        return;
    }
    const uint64_t b = gb - pr.block_off;
    if (b >= d.L.nblocks) return;  // blocks of an empty pair's neighbours
    d.begin = 0;
    d.end = lp.n;
    d.raw_cap = raw_cap;
    d.bytes = lp.blob_cap;
    d.flags = stats;
    decode_block<KB, true>(blob + lp.blob_off, d, b, raw_cap, reinterpret_cast<uint8_t*>(keys) + pr.key_off * KB);
}

// flag[i] = probe key i is the first copy of its value within its pair and
// the pair's target list (compressed) holds it.
template <int KB>
__global__ __launch_bounds__(kSetTile) void pair_flags_kernel(const uint8_t* __restrict__ blob,
                                                              const lc_batch_list* __restrict__ lists, BatchArgs a,
                                                              const lc_list_pair* __restrict__ pairs, uint32_t npairs,
                                                              uint64_t total_keys, uint64_t total_blocks,
                                                              const void* __restrict__ keys,
                                                              uint8_t* __restrict__ flags, uint64_t* __restrict__ cnt,
                                                              uint64_t tile0)
{
    const uint64_t tile = tile0 + blockIdx.x;
    const uint64_t i = tile * kSetTile + threadIdx.x;
    uint32_t f = 0;
    if (i < total_keys) {
        const lc_list_pair pr = pairs[find_pair<false>(pairs, npairs, i)];
        lc_batch_list lp, lt;
        Layout Lp, Lt;
        if (pair_fits(pr, lists, a, total_keys, total_blocks, &lp, &lt, &Lp, &Lt) && i - pr.key_off < pr.n) {
            const uint64_t x = load_key<KB>(keys, i);
            f = (i == pr.key_off || load_key<KB>(keys, i - 1) != x) && contains_one<KB>(blob + lt.blob_off, Lt, x);
        }
        flags[i] = (uint8_t)f;
    }
    tile_count(f, cnt, tile);
}

// Found keys packed at the start of their pair's region; counts per pair.
template <int KB>
__global__ __launch_bounds__(kSetTile) void pair_scatter_kernel(const lc_list_pair* __restrict__ pairs,
                                                                uint32_t npairs, uint64_t total_keys,
                                                                const void* __restrict__ keys,
                                                                const uint8_t* __restrict__ flags,
                                                                const uint64_t* __restrict__ P, void* __restrict__ out,
                                                                uint64_t tile0)
{
    const uint64_t i = (tile0 + blockIdx.x) * kSetTile + threadIdx.x;
    if (i >= total_keys || !flags[i]) return;
    const lc_list_pair pr = pairs[find_pair<false>(pairs, npairs, i)];
    store_key<KB>(out, pr.key_off + (P[i] - P[pr.key_off]), load_key<KB>(keys, i));
}

__global__ __launch_bounds__(256) void pair_counts_kernel(const lc_list_pair* __restrict__ pairs, uint32_t npairs,
                                                          uint64_t total_keys, const uint64_t* __restrict__ P,
                                                          uint64_t* __restrict__ counts)
{
    const uint32_t p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npairs) return;
    const lc_list_pair pr = pairs[p];
    const bool ok = pr.key_off <= total_keys && pr.n <= total_keys - pr.key_off;
    counts[p] = ok ? P[pr.key_off + pr.n] - P[pr.key_off] : 0;
}

// eps of list l := the candidate with the smallest size (ties: the smaller
// eps, i.e. the earlier candidate).
__global__ __launch_bounds__(256) void batch_pick_kernel(lc_batch_list* __restrict__ lists, uint32_t nlists,
                                                         const uint64_t* __restrict__ sizes, Cands cands)
{
    const uint32_t l = blockIdx.x * 256 + threadIdx.x;
    if (l >= nlists) return;
    uint32_t best = 0;
    for (uint32_t c = 1; c < cands.n; c++)
        if (sizes[(uint64_t)c * nlists + l] < sizes[(uint64_t)best * nlists + l]) best = c;
    lists[l].eps = cands.eps[best];
}

// kernel over `tiles` tiles of kSetTile threads, at most kMaxGrid per launch
template <typename Fn>
void over_tiles(uint64_t tiles, Fn launch)
{
    for (uint64_t t0 = 0; t0 < tiles; t0 += kMaxGrid) launch((uint32_t)(tiles - t0 < kMaxGrid ? tiles - t0 : kMaxGrid), t0);
}

// Point-query launches: one query per thread up to 2^24 queries (the
// kernels loop beyond that).  Many short workgroups, replaced as they finish,
// beat a grid that fills the chip once with long per-thread loops: 1e7
// random access(i) ran 3 % faster on a 608 MB blob and 2 % on a 120 MB one.
inline uint32_t query_grid(uint64_t m)
{
    const uint64_t g = (m + 255) / 256;
    return (uint32_t)(g < 65536 ? (g ? g : 1) : 65536);
}


// Raises kernel f's dynamic LDS limit to `bytes` (above the default 64 KB)
// once per device; later calls with no larger need make no runtime call, so
// launches stay capturable into graphs.
hipError_t allow_lds(const void* f, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    struct Entry {
        const void* f;
        int dev;
        size_t bytes;
    };
    static std::mutex mu;
    static Entry set[64];
    static int nset = 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < nset; i++)
        if (set[i].f == f && set[i].dev == dev && set[i].bytes >= bytes) return hipSuccess;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    for (int i = 0; i < nset; i++)
        if (set[i].f == f && set[i].dev == dev) {
            set[i].bytes = bytes;
            return hipSuccess;
        }
    if (nset < 64) set[nset++] = Entry{f, dev, bytes};
    return hipSuccess;
}

hipError_t launch_batch_fit(const void* d_keys, const lc_batch_list* d_lists, const BatchArgs& a, const Cands& c,
                            uint8_t* d_blob, const Workspace& ws, uint64_t* d_sizes, uint32_t* d_stats, bool sizes_only,
                            hipStream_t stream)
{
    const uint32_t ncand = sizes_only ? c.n : 1u;
    uint32_t eps_max = 0;
    for (uint32_t k = 0; k < (sizes_only ? c.n : 0u); k++) eps_max = c.eps[k] > eps_max ? c.eps[k] : eps_max;
    if (!sizes_only) eps_max = a.max_eps;
    uint32_t w = 0;
    while ((1ull << w) < 2ull * eps_max + 1) w++;
    const uint64_t res_stride = align16(((1ull << a.log2b) * w + 7) / 8);
    const bool lanes = a.tiling == LC_TILING_LANES || (a.tiling == LC_TILING_AUTO && a.total_blocks >= kLanesMinBlocks);
    if (a.fit == LC_FIT_MIN || a.fit == LC_FIT_OPT) {
        const uint64_t B = 1ull << a.log2b;
        const size_t lds = a.fit == LC_FIT_OPT
                               ? a.kb * B + res_stride + 16 + 4 * B
                               : 16 + a.kb * B + res_stride + 16 + align16(2 * B) + align16(2 * (B + 1));
        auto k = a.kb == 4 ? (sizes_only ? batch_block_fit_kernel<4, true, LC_FIT_MIN>
                                         : batch_block_fit_kernel<4, false, LC_FIT_MIN>)
                           : (sizes_only ? batch_block_fit_kernel<8, true, LC_FIT_MIN>
                                         : batch_block_fit_kernel<8, false, LC_FIT_MIN>);
        if (a.fit == LC_FIT_OPT)
            k = a.kb == 4 ? (sizes_only ? batch_block_fit_kernel<4, true, LC_FIT_OPT>
                                        : batch_block_fit_kernel<4, false, LC_FIT_OPT>)
                          : (sizes_only ? batch_block_fit_kernel<8, true, LC_FIT_OPT>
                                        : batch_block_fit_kernel<8, false, LC_FIT_OPT>);
        const hipError_t e = allow_lds((const void*)k, lds);
        if (e != hipSuccess) return e;
        const uint64_t items = a.total_blocks * ncand;
        for (uint64_t i0 = 0; i0 < items; i0 += kMaxGrid) {
            const uint64_t g = items - i0 < kMaxGrid ? items - i0 : kMaxGrid;
            hipLaunchKernelGGL(k, dim3((uint32_t)g), dim3(64), lds, stream, d_keys, d_lists, a, c, d_blob, ws, d_stats,
                               i0);
        }
    } else if (lanes) {
        const uint64_t items = (a.total_blocks + 63) / 64 * ncand;
        auto k = a.kb == 4 ? (sizes_only ? batch_lanes_kernel<4, true> : batch_lanes_kernel<4, false>)
                           : (sizes_only ? batch_lanes_kernel<8, true> : batch_lanes_kernel<8, false>);
        for (uint64_t i0 = 0; i0 < items; i0 += kMaxGrid) {
            const uint64_t g = items - i0 < kMaxGrid ? items - i0 : kMaxGrid;
            hipLaunchKernelGGL(k, dim3((uint32_t)g), dim3(64), lane_fit_lds(a.log2b), stream, d_keys, d_lists, a, c,
                               d_blob, ws, d_stats, i0);
        }
        if (!sizes_only) {
            auto kc = a.kb == 4 ? batch_code_pack_kernel<4> : batch_code_pack_kernel<8>;
            const size_t clds = code_pack_lds(a.log2b, res_stride);
            for (uint64_t b0 = 0; b0 < a.total_blocks; b0 += kMaxGrid) {
                const uint64_t nw = a.total_blocks - b0 < kMaxGrid ? a.total_blocks - b0 : kMaxGrid;
                hipLaunchKernelGGL(kc, dim3((uint32_t)nw), dim3(64), clds, stream, d_keys, d_lists, a, d_blob, ws, b0);
            }
        }
    } else {
        const size_t lds = 4 * (res_stride + 16);
        const uint64_t items = a.total_groups * ncand;
        auto k = a.kb == 4 ? (sizes_only ? batch_fit_kernel<4, true> : batch_fit_kernel<4, false>)
                           : (sizes_only ? batch_fit_kernel<8, true> : batch_fit_kernel<8, false>);
        for (uint64_t i0 = 0; i0 < items; i0 += kMaxGrid) {
            const uint64_t g = items - i0 < kMaxGrid ? items - i0 : kMaxGrid;
            hipLaunchKernelGGL(k, dim3((uint32_t)g), dim3(64), lds, stream, d_keys, d_lists, a, c, d_blob, ws, d_stats,
                               i0);
        }
    }
    const uint64_t scans = (uint64_t)a.nlists * ncand;
    auto ks = sizes_only ? batch_scan_kernel<true> : batch_scan_kernel<false>;
    for (uint64_t i0 = 0; i0 < scans; i0 += kMaxGrid) {
        const uint64_t g = scans - i0 < kMaxGrid ? scans - i0 : kMaxGrid;
        hipLaunchKernelGGL(ks, dim3((uint32_t)g), dim3(256), 0, stream, d_lists, a, c, d_blob, ws, d_sizes, d_stats, i0);
    }
    if (!sizes_only) {
        constexpr uint64_t per = 256 / kEmitLanes;
        const uint64_t groups = (a.total_blocks + per - 1) / per;
        for (uint64_t g0 = 0; g0 < groups; g0 += kMaxGrid) {
            const uint64_t g = groups - g0 < kMaxGrid ? groups - g0 : kMaxGrid;
            hipLaunchKernelGGL(batch_emit_kernel, dim3((uint32_t)g), dim3(256), 0, stream, d_lists, a, d_blob, ws,
                               g0 * per);
        }
    }
    return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_batch_compress(const void* d_keys, const lc_batch_list* d_lists, const BatchArgs& a, const uint32_t* cands,
                                 uint32_t ncand, uint8_t* d_blob, const Workspace& ws, uint64_t* d_sizes,
                                 uint32_t* d_stats, bool sizes_only, hipStream_t stream)
{
    Cands c{};
    c.n = ncand;
    for (uint32_t k = 0; k < ncand && k < kMaxCands; k++) c.eps[k] = cands[k];
    return launch_batch_fit(d_keys, d_lists, a, c, d_blob, ws, d_sizes, d_stats, sizes_only, stream);
}

hipError_t launch_batch_pick(lc_batch_list* d_lists, uint32_t nlists, const uint64_t* d_sizes, const uint32_t* cands,
                             uint32_t ncand, hipStream_t stream)
{
    Cands c{};
    c.n = ncand;
    for (uint32_t k = 0; k < ncand && k < kMaxCands; k++) c.eps[k] = cands[k];
    hipLaunchKernelGGL(batch_pick_kernel, dim3((nlists + 255) / 256), dim3(256), 0, stream, d_lists, nlists, d_sizes, c);
    return hipGetLastError();
}

hipError_t launch_batch_decode(const uint8_t* d_blob, const lc_batch_list* d_lists, const BatchArgs& a,
                               uint32_t max_seg_bytes, void* d_out, uint32_t* d_stats, hipStream_t stream)
{
    if (a.total_blocks == 0) return hipSuccess;
    uint32_t w = 0;
    while ((1ull << w) < 2ull * a.max_eps + 1) w++;
    const uint64_t res_stride = align16(((1ull << a.log2b) * w + 7) / 8);
    const uint32_t raw_cap = decode_raw_cap(max_seg_bytes, kSegRawSmall);
    const size_t lds = decode_lds_bytes(a.log2b, res_stride, raw_cap);
    auto k = a.kb == 4 ? batch_decode_kernel<4> : batch_decode_kernel<8>;
    hipError_t e = allow_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    for (uint64_t b0 = 0; b0 < a.total_blocks; b0 += kMaxGrid) {
        const uint64_t nblk = a.total_blocks - b0 < kMaxGrid ? a.total_blocks - b0 : kMaxGrid;
        const uint64_t per_xcd = (nblk + 7) / 8;
        hipLaunchKernelGGL(k, dim3((uint32_t)(per_xcd * 8)), dim3(64), lds, stream, d_blob, d_lists, a, b0, nblk,
                           per_xcd, raw_cap, d_out, d_stats);
    }
    return hipGetLastError();
}

hipError_t launch_batch_and(const uint8_t* d_blob, const lc_batch_list* d_lists, const BatchArgs& a,
                            const lc_list_pair* d_pairs, uint32_t npairs, uint64_t total_keys, uint64_t total_blocks,
                            uint32_t max_seg_bytes, const PairWs& w, void* d_out, uint64_t* d_counts,
                            uint32_t* d_stats, hipStream_t stream)
{
    uint32_t wd = 0;
    while ((1ull << wd) < 2ull * a.max_eps + 1) wd++;
    const uint64_t res_stride = align16(((1ull << a.log2b) * wd + 7) / 8);
    const uint32_t raw_cap = decode_raw_cap(max_seg_bytes, kSegRawSmall);
    const size_t lds = decode_lds_bytes(a.log2b, res_stride, raw_cap);
    auto kd = a.kb == 4 ? pair_decode_kernel<4> : pair_decode_kernel<8>;
    hipError_t e = allow_lds((const void*)kd, lds);
    if (e != hipSuccess) return e;
    for (uint64_t b0 = 0; b0 < total_blocks; b0 += kMaxGrid) {
        const uint64_t nblk = total_blocks - b0 < kMaxGrid ? total_blocks - b0 : kMaxGrid;
        const uint64_t per_xcd = (nblk + 7) / 8;
        hipLaunchKernelGGL(kd, dim3((uint32_t)(per_xcd * 8)), dim3(64), lds, stream, d_blob, d_lists, a, d_pairs,
                           npairs, total_keys, total_blocks, b0, nblk, per_xcd, raw_cap, w.keys, d_stats);
    }
    const uint64_t tiles = (total_keys + kSetTile - 1) / kSetTile;
    auto kf = a.kb == 4 ? pair_flags_kernel<4> : pair_flags_kernel<8>;
    over_tiles(tiles, [&](uint32_t g, uint64_t t0) {
        hipLaunchKernelGGL(kf, dim3(g), dim3(kSetTile), 0, stream, d_blob, d_lists, a, d_pairs, npairs, total_keys,
                           total_blocks, w.keys, w.flags, w.cnt, t0);
    });
    hipLaunchKernelGGL(set_tiles_scan_kernel, dim3(1), dim3(1024), 0, stream, w.cnt, tiles, (uint64_t)0, w.tot,
                       w.tot + 1);
    over_tiles(total_keys / kSetTile + 1, [&](uint32_t g, uint64_t t0) {
        hipLaunchKernelGGL(prefix_kernel, dim3(g), dim3(kSetTile), 0, stream, w.flags, total_keys, w.cnt, w.tot, w.P,
                           t0);
    });
    auto ks = a.kb == 4 ? pair_scatter_kernel<4> : pair_scatter_kernel<8>;
    over_tiles(tiles, [&](uint32_t g, uint64_t t0) {
        hipLaunchKernelGGL(ks, dim3(g), dim3(kSetTile), 0, stream, d_pairs, npairs, total_keys, w.keys, w.flags, w.P,
                           d_out, t0);
    });
    hipLaunchKernelGGL(pair_counts_kernel, dim3((npairs + 255) / 256), dim3(256), 0, stream, d_pairs, npairs,
                       total_keys, w.P, d_counts);
    return hipGetLastError();
}

hipError_t launch_compress(const void* d_keys, const Layout& L, uint32_t fit, uint8_t* d_blob, const Workspace& ws,
                           uint64_t* d_blob_bytes, uint32_t* d_flags, hipStream_t stream)
{
    bool lanes = false;
    if (L.nblocks && fit == LC_FIT_OPT) {
        const uint64_t B = 1ull << L.log2b;
        const size_t lds = L.kb * B + L.res_stride + 16 + 4 * B;
        auto k = L.kb == 4 ? fit_opt_kernel<4> : fit_opt_kernel<8>;
        const hipError_t e = allow_lds((const void*)k, lds);
        if (e != hipSuccess) return e;
        for (uint64_t b0 = 0; b0 < L.nblocks; b0 += kMaxGrid) {
            const uint64_t nw = L.nblocks - b0 < kMaxGrid ? L.nblocks - b0 : kMaxGrid;
            hipLaunchKernelGGL(k, dim3((uint32_t)nw), dim3(64), lds, stream, d_keys, L, d_blob, ws, d_flags, b0);
        }
    } else if (L.nblocks && fit == LC_FIT_MIN) {
        const uint64_t B = 1ull << L.log2b;
        const size_t lds = 16 + L.kb * B + L.res_stride + 16 + align16(2 * B) + align16(2 * (B + 1));
        auto k = L.kb == 4 ? fit_min_kernel<4> : fit_min_kernel<8>;
        const hipError_t e = allow_lds((const void*)k, lds);
        if (e != hipSuccess) return e;
        for (uint64_t b0 = 0; b0 < L.nblocks; b0 += kMaxGrid) {
            const uint64_t nw = L.nblocks - b0 < kMaxGrid ? L.nblocks - b0 : kMaxGrid;
            hipLaunchKernelGGL(k, dim3((uint32_t)nw), dim3(kMinLanes), lds, stream, d_keys, L, d_blob, ws, d_flags,
                               b0);
        }
    } else if (L.nblocks >= kLanesMinBlocks) {
        auto kf = L.kb == 4 ? fit_lanes_kernel<4> : fit_lanes_kernel<8>;
        const uint64_t waves = (L.nblocks + 63) / 64;
        for (uint64_t g0 = 0; g0 < waves; g0 += kMaxGrid) {
            const uint64_t ng = waves - g0 < kMaxGrid ? waves - g0 : kMaxGrid;
            hipLaunchKernelGGL(kf, dim3((uint32_t)ng), dim3(64), lane_fit_lds(L.log2b), stream, d_keys, L, d_blob, ws,
                               d_flags, g0 * 64);
        }
        // the codes and the segment areas come after the directory (code_pack_kernel)
        lanes = true;
    } else if (L.nblocks) {
        const size_t lds = 4 * (L.res_stride + 16);
        auto k = L.kb == 4 ? fit_pack_kernel<4> : fit_pack_kernel<8>;
        const uint64_t groups = (L.nblocks + 3) / 4;
        for (uint64_t g0 = 0; g0 < groups; g0 += kMaxGrid) {
            const uint64_t ng = groups - g0 < kMaxGrid ? groups - g0 : kMaxGrid;
            hipLaunchKernelGGL(k, dim3((uint32_t)ng), dim3(64), lds, stream, d_keys, L, d_blob, ws, d_flags, g0 * 4);
        }
    }
    if (L.nblocks) {
        const uint64_t nt = ntiles_of(L.nblocks);
        for (uint64_t t0 = 0; t0 < nt; t0 += kMaxGrid) {
            const uint64_t g = nt - t0 < kMaxGrid ? nt - t0 : kMaxGrid;
            hipLaunchKernelGGL(tile_reduce_kernel, dim3((uint32_t)g), dim3(256), 0, stream, ws, L.nblocks, t0);
        }
    }
    hipLaunchKernelGGL(tile_scan_kernel, dim3(1), dim3(1024), 0, stream, ws, L, d_blob, d_blob_bytes);
    if (L.nblocks) {
        const uint64_t nt = ntiles_of(L.nblocks);
        for (uint64_t t0 = 0; t0 < nt; t0 += kMaxGrid) {
            const uint64_t g = nt - t0 < kMaxGrid ? nt - t0 : kMaxGrid;
            hipLaunchKernelGGL(dir_emit_kernel, dim3((uint32_t)g), dim3(256), 0, stream, ws, L, d_blob, t0);
        }
        if (lanes) {
            const size_t lds = code_pack_lds(L.log2b, L.res_stride);
            auto kc = L.kb == 4 ? code_pack_kernel<4> : code_pack_kernel<8>;
            for (uint64_t b0 = 0; b0 < L.nblocks; b0 += kMaxGrid) {
                const uint64_t nw = L.nblocks - b0 < kMaxGrid ? L.nblocks - b0 : kMaxGrid;
                hipLaunchKernelGGL(kc, dim3((uint32_t)nw), dim3(64), lds, stream, d_keys, L, d_blob, ws, b0);
            }
        } else {
            constexpr uint64_t per = 256 / kEmitLanes;
            const uint64_t egroups = (L.nblocks + per - 1) / per;
            for (uint64_t g0 = 0; g0 < egroups; g0 += kMaxGrid) {
                const uint64_t g = egroups - g0 < kMaxGrid ? egroups - g0 : kMaxGrid;
                hipLaunchKernelGGL(seg_emit_kernel, dim3((uint32_t)g), dim3(256), 0, stream, ws, L, d_blob,
                                   g0 * per);
            }
        }
    }
    return hipGetLastError();
}

hipError_t launch_decode(const uint8_t* d_blob, const Layout& L, uint64_t begin, uint64_t end, void* d_out,
                         hipStream_t stream, bool approx)
{
    if (begin >= end) return hipSuccess;
    const uint64_t b_lo = begin >> L.log2b, b_hi = (end - 1) >> L.log2b;
    const uint32_t raw_cap = decode_raw_cap(L.max_seg_bytes, kSegRawSmall);
    const size_t lds = decode_lds_bytes(L.log2b, L.res_stride, raw_cap);
    const bool range = approx || !(begin == 0 && end == L.n);
    auto k = L.kb == 4 ? (approx ? decode_kernel<4, true, true> : range ? decode_kernel<4, true> : decode_kernel<4, false>)
                       : (approx ? decode_kernel<8, true, true> : range ? decode_kernel<8, true> : decode_kernel<8, false>);
    hipError_t e = allow_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    // A decode (full or range) stages the compressed bytes of its blocks in
    // the on-die cache from inside its own launch (decode_full_kernel; T a
    // multiple of 8 keeps the XCD-major block order).  Otherwise a separate
    // pass stages the bytes the decode will read: the whole tail of the blob
    // for a full decode past the grid limit; the directory entries and slabs
    // of the blocks touched for such a range (its segment areas are found
    // only through the directory); the directory entries and segment areas
    // for the approximate decode, which reads no slab.
    const uint64_t nblk = b_hi + 1 - b_lo;
    if (!approx && nblk <= kMaxGrid - kStreamGroups) {
        auto kf = L.kb == 4 ? (range ? decode_full_kernel<4, true> : decode_full_kernel<4, false>)
                            : (range ? decode_full_kernel<8, true> : decode_full_kernel<8, false>);
        e = allow_lds((const void*)kf, lds);
        if (e != hipSuccess) return e;
        const uint64_t nch = (nblk + kStreamChunk - 1) / kStreamChunk;
        const uint32_t T = (uint32_t)((nch < kStreamGroups ? nch : kStreamGroups) + 7) / 8 * 8;
        DecodeArgs a;
        a.L = L;
        a.begin = begin;
        a.end = end;
        a.b_first = b_lo;
        a.nblk = nblk;
        a.per_xcd = (a.nblk + 7) / 8;
        a.raw_cap = raw_cap;
        a.bytes = L.blob_bytes;
        a.flags = nullptr;
        hipLaunchKernelGGL(kf, dim3((uint32_t)(T + a.per_xcd * 8)), dim3(64), lds, stream, d_blob, a, T, d_out);
        return hipGetLastError();
    }
    if (approx) {
        if (b_hi + 1 - b_lo >= kTouchMinBytes / 1024)
            hipLaunchKernelGGL(touch_blocks_kernel, dim3(kTouchGrid), dim3(256), 0, stream, d_blob, L, b_lo, b_hi);
    } else if (!range) {
        hipLaunchKernelGGL(touch_kernel, dim3(kTouchGrid), dim3(256), 0, stream, d_blob, L.off_dir, L.blob_bytes);
    } else {
        const uint64_t d_lo = L.off_dir + 16 * b_lo, d_hi = L.off_dir + 16 * (b_hi + 1);
        const uint64_t r_lo = L.off_res + b_lo * L.res_stride, r_hi = L.off_res + (b_hi + 1) * L.res_stride;
        if (d_hi - d_lo + r_hi - r_lo >= kTouchMinBytes) {
            hipLaunchKernelGGL(touch_kernel, dim3(kTouchGrid), dim3(256), 0, stream, d_blob, d_lo, d_hi);
            hipLaunchKernelGGL(touch_kernel, dim3(kTouchGrid), dim3(256), 0, stream, d_blob, r_lo, r_hi);
        }
    }
    for (uint64_t b0 = b_lo; b0 <= b_hi; b0 += kMaxGrid) {
        DecodeArgs a;
        a.L = L;
        a.begin = begin;
        a.end = end;
        a.b_first = b0;
        a.nblk = (b_hi + 1 - b0) < kMaxGrid ? (b_hi + 1 - b0) : kMaxGrid;
        a.per_xcd = (a.nblk + 7) / 8;
        a.raw_cap = raw_cap;
        a.bytes = L.blob_bytes;
        a.flags = nullptr;
        hipLaunchKernelGGL(k, dim3((uint32_t)(a.per_xcd * 8)), dim3(64), lds, stream, d_blob, a, d_out);
    }
    return hipGetLastError();
}

hipError_t launch_quantile(const uint8_t* d_blob, const Layout& L, const uint64_t* d_k, uint64_t q, uint64_t m,
                           bool approx, void* d_out, hipStream_t stream)
{
    if (m == 0) return hipSuccess;
    auto k = L.kb == 4 ? (approx ? quantile_kernel<4, true> : quantile_kernel<4, false>)
                       : (approx ? quantile_kernel<8, true> : quantile_kernel<8, false>);
    hipLaunchKernelGGL(k, dim3(query_grid(m)), dim3(256), 0, stream, d_blob, L, d_k, q, m, d_out);
    return hipGetLastError();
}

namespace {

template <int KB>
hipError_t setop_impl(uint32_t op, const uint8_t* blob_a, const Layout& La, const uint8_t* blob_b, const Layout& Lb,
                      const SetWs& w, void* out, uint64_t* count, hipStream_t st)
{
    hipError_t e = hipSuccess;
    const uint64_t na = La.n, nb = Lb.n;
    const uint64_t ta = (na + kSetTile - 1) / kSetTile, tb = (nb + kSetTile - 1) / kSetTile;
    if (na && (e = launch_decode(blob_a, La, 0, na, w.a_keys, st)) != hipSuccess) return e;
    if (op == LC_SETOP_INTERSECT) {
        over_tiles(ta, [&](uint32_t g, uint64_t t0) {
            hipLaunchKernelGGL(and_flags_kernel<KB>, dim3(g), dim3(kSetTile), 0, st, blob_b, Lb, w.a_keys, na, w.fa,
                               w.cnt, t0);
        });
        hipLaunchKernelGGL(set_tiles_scan_kernel, dim3(1), dim3(1024), 0, st, w.cnt, ta, (uint64_t)0, w.tot, count);
        over_tiles(ta, [&](uint32_t g, uint64_t t0) {
            hipLaunchKernelGGL(and_scatter_kernel<KB>, dim3(g), dim3(kSetTile), 0, st, w.a_keys, na, w.fa, w.cnt, out,
                               t0);
        });
        return hipGetLastError();
    }
    if (nb && (e = launch_decode(blob_b, Lb, 0, nb, w.b_keys, st)) != hipSuccess) return e;
    over_tiles(ta + tb, [&](uint32_t g, uint64_t t0) {
        hipLaunchKernelGGL(or_flags_kernel<KB>, dim3(g), dim3(kSetTile), 0, st, w.a_keys, na, w.b_keys, nb, ta, w.fa,
                           w.fb, w.cnt, t0);
    });
    hipLaunchKernelGGL(set_tiles_scan_kernel, dim3(1), dim3(1024), 0, st, w.cnt, ta, tb, w.tot, count);
    over_tiles(na / kSetTile + 1, [&](uint32_t g, uint64_t t0) {
        hipLaunchKernelGGL(prefix_kernel, dim3(g), dim3(kSetTile), 0, st, w.fa, na, w.cnt, w.tot, w.PA, t0);
    });
    over_tiles(nb / kSetTile + 1, [&](uint32_t g, uint64_t t0) {
        hipLaunchKernelGGL(prefix_kernel, dim3(g), dim3(kSetTile), 0, st, w.fb, nb, w.cnt + ta, w.tot + 1, w.PB, t0);
    });
    over_tiles(ta + tb, [&](uint32_t g, uint64_t t0) {
        hipLaunchKernelGGL(or_scatter_kernel<KB>, dim3(g), dim3(kSetTile), 0, st, w.a_keys, na, w.b_keys, nb, ta, w.fa,
                           w.fb, w.PA, w.PB, out, t0);
    });
    return hipGetLastError();
}

}  // namespace

hipError_t launch_setop(uint32_t op, const uint8_t* blob_a, const Layout& La, const uint8_t* blob_b, const Layout& Lb,
                        const SetWs& w, void* out, uint64_t* count, hipStream_t stream)
{
    return La.kb == 4 ? setop_impl<4>(op, blob_a, La, blob_b, Lb, w, out, count, stream)
                      : setop_impl<8>(op, blob_a, La, blob_b, Lb, w, out, count, stream);
}

hipError_t launch_serve(const uint8_t* d_blob, const ServeArgs& args, const ServeRange* d_ranges,
                        const ServePoint* d_points, uint8_t* d_arena, hipStream_t stream)
{
    ServeArgs s = args;
    // areas above the small cap decode from global memory (decode_segments)
    s.raw_cap = decode_raw_cap(s.L.max_seg_bytes, kSegRawSmall);
    const uint64_t waves = s.range_items + (s.npoint + 63) / 64;
    if (waves == 0) return hipSuccess;
    auto k = s.L.kb == 4 ? serve_kernel<4> : serve_kernel<8>;
    const size_t lds = decode_lds_bytes(s.L.log2b, s.L.res_stride, s.raw_cap);
    hipError_t e = allow_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3((uint32_t)waves), dim3(64), lds, stream, d_blob, s, d_ranges, d_points, d_arena);
    return hipGetLastError();
}

hipError_t launch_access(const uint8_t* d_blob, const Layout& L, const uint64_t* d_idx, uint64_t m, void* d_out,
                         uint32_t* d_flags, hipStream_t stream)
{
    if (m == 0) return hipSuccess;
    auto k = L.kb == 4 ? access_kernel<4> : access_kernel<8>;
    hipLaunchKernelGGL(k, dim3(query_grid(m)), dim3(256), 0, stream, d_blob, L, d_idx, m, d_out, d_flags);
    return hipGetLastError();
}

hipError_t launch_lower_bound(const uint8_t* d_blob, const Layout& L, const void* d_q, uint64_t m, uint64_t* d_pos,
                              hipStream_t stream)
{
    if (m == 0) return hipSuccess;
    auto k = L.kb == 4 ? lower_bound_kernel<4> : lower_bound_kernel<8>;
    hipLaunchKernelGGL(k, dim3(query_grid(m)), dim3(256), 0, stream, d_blob, L, d_q, m, d_pos);
    return hipGetLastError();
}

}  // namespace lc
