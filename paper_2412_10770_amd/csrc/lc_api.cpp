// C ABI of the learned compressor (declared in include/lc.h): argument
// checks, blob layout, workspace carving and kernel launches.  All checks that
// can fail happen before anything is enqueued.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <utility>

#include "lc.h"
#include "lc_launch.h"

#define LC_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr uint64_t kMaxKeys = 1ull << 40;
constexpr uint32_t kMagic = 0x3142434Cu;

// Residual width: the smallest w with 2^w >= 2 eps + 1.
uint32_t residual_width(uint32_t eps)
{
    const uint64_t span = 2ull * eps + 1;
    uint32_t w = 0;
    while ((1ull << w) < span) w++;
    return w;
}

lc_status check_params(const lc_params* p)
{
    if (!p) return LC_EINVAL;
    if (p->key_bytes != 4 && p->key_bytes != 8) return LC_EINVAL;
    if (p->log2_block < 6 || p->log2_block > 12) return LC_EINVAL;
    if (p->frac_bits > 32 || p->fit > LC_FIT_OPT) return LC_EINVAL;
    if (p->eps > LC_MAX_EPS) return LC_EINVAL;
    return LC_OK;
}

// Fixed part of the layout (everything but the segment areas).
lc::Layout fixed_layout(uint64_t n, const lc_params* p)
{
    lc::Layout L{};
    const uint64_t B = 1ull << p->log2_block;
    L.n = n;
    L.nblocks = (n + B - 1) / B;
    L.kb = p->key_bytes;
    L.log2b = p->log2_block;
    L.F = p->frac_bits;
    L.eps = p->eps;
    L.w = residual_width(p->eps);
    L.res_stride = lc::align16((B * L.w + 7) / 8);
    L.off_first = lc::kHeaderBytes;
    L.off_dir = L.off_first + lc::align16(L.nblocks * L.kb);
    L.off_res = L.off_dir + 16 * L.nblocks;
    L.off_seg = L.off_res + L.nblocks * L.res_stride;
    L.max_nseg = 0;
    L.flags = p->fit == LC_FIT_OPT ? lc::kFlagFrac : 0u;
    L.fb = L.flags ? lc::frac_bytes(L.F) : 0u;
    return L;
}

struct WsPlan {
    uint64_t blk, tiles, start, delta, slope, frac, total;
};

WsPlan plan_workspace(const lc::Layout& L)
{
    const uint64_t recs = L.nblocks << L.log2b;
    WsPlan w;
    w.blk = 0;
    w.tiles = w.blk + lc::align16(L.nblocks * sizeof(lc::BlockInfo));
    w.start = w.tiles + lc::align16(lc::ntiles_of(L.nblocks) * sizeof(lc::TileSum));
    w.delta = w.start + lc::align16(recs * 2);
    w.slope = w.delta + recs * 8;
    w.frac = w.slope + recs * 8;
    w.total = w.frac + (L.flags ? recs * 4 : 0);
    if (w.total == 0) w.total = 16;
    return w;
}

uint64_t worst_blob(const lc::Layout& L)
{
    const uint64_t B = 1ull << L.log2b;
    const uint64_t seg_area = lc::align16(2 * B) + 2 * lc::align16(8 * B) + lc::align16(L.fb * B);
    return L.off_seg + L.nblocks * seg_area;
}

uint64_t rd(const uint8_t* p, int nbytes)
{
    uint64_t v = 0;
    for (int i = 0; i < nbytes; i++) v |= (uint64_t)p[i] << (8 * i);
    return v;
}

// Layout of a parsed blob, re-checked (the info struct comes from the caller).
lc_status layout_of(const lc_blob_info* info, lc::Layout* L)
{
    if (!info) return LC_EINVAL;
    lc_params p{};
    p.key_bytes = (uint8_t)info->key_bytes;
    p.log2_block = (uint8_t)info->log2_block;
    p.frac_bits = (uint8_t)info->frac_bits;
    p.eps = info->eps;
    if (info->flags & ~lc::kFlagFrac) return LC_EINVAL;
    p.fit = info->flags ? LC_FIT_OPT : LC_FIT_GREEDY;  // the layout depends on it only through the fractions
    if (info->key_bytes > 8 || info->log2_block > 12 || info->frac_bits > 32) return LC_EINVAL;
    if (check_params(&p) != LC_OK || info->n > kMaxKeys) return LC_EINVAL;
    *L = fixed_layout(info->n, &p);
    if (L->w != info->width || L->nblocks != info->nblocks || L->off_first != info->off_first ||
        L->off_dir != info->off_dir || L->off_res != info->off_res || L->res_stride != info->res_stride ||
        L->off_seg != info->off_seg)
        return LC_EINVAL;
    const uint64_t B = 1ull << info->log2_block;
    if (info->n && (info->max_nseg == 0 || info->max_nseg > B)) return LC_EINVAL;
    if (info->blob_bytes < L->off_seg) return LC_EINVAL;
    if (info->n && (info->max_seg_bytes < 48 ||
                    info->max_seg_bytes > lc::align16(2 * B) + 2 * lc::align16(8 * B) + lc::align16(L->fb * B) ||
                    info->max_seg_bytes % 16))
        return LC_EINVAL;
    L->max_nseg = info->max_nseg;
    L->max_seg_bytes = info->max_seg_bytes;
    L->blob_bytes = info->blob_bytes;
    return LC_OK;
}

constexpr uint64_t kBlockInfoBytes = sizeof(lc::BlockInfo);

lc_status check_batch(const lc_batch_params* p)
{
    if (!p || p->nlists == 0 || p->tiling > LC_TILING_LANES || p->fit > LC_FIT_OPT) return LC_EINVAL;
    lc_params q{};
    q.key_bytes = p->key_bytes;
    q.log2_block = p->log2_block;
    q.frac_bits = p->frac_bits;
    q.fit = (uint8_t)p->fit;
    q.eps = p->max_eps;
    return check_params(&q);
}

// Batch workspace: block infos for up to LC_BATCH_MAX_CANDIDATES size passes,
// then the segment records of every block (start, anchor delta, slope, and
// the intercept fraction with the optimal fit).
struct BatchWs {
    uint64_t blk, start, delta, slope, frac, total;
};

BatchWs plan_batch_ws(uint64_t total_blocks, uint32_t log2b, uint32_t fit)
{
    const uint64_t recs = total_blocks << log2b;
    BatchWs w;
    w.blk = 0;
    w.start = lc::align16(LC_BATCH_MAX_CANDIDATES * total_blocks * kBlockInfoBytes);
    w.delta = w.start + lc::align16(recs * 2);
    w.slope = w.delta + recs * 8;
    w.frac = w.slope + recs * 8;
    w.total = w.frac + (fit == LC_FIT_OPT ? recs * 4 : 0);
    if (w.total == 0) w.total = 16;
    return w;
}

lc::BatchArgs batch_args(const lc_batch_params* p, uint64_t nkeys, uint64_t blob_cap)
{
    lc::BatchArgs a{};
    a.kb = p->key_bytes;
    a.log2b = p->log2_block;
    a.F = p->frac_bits;
    a.nlists = p->nlists;
    a.max_eps = p->max_eps;
    a.tiling = p->tiling;
    a.fit = p->fit;
    a.total_blocks = p->total_blocks;
    a.total_groups = p->total_groups;
    a.nkeys = nkeys;
    a.blob_cap = blob_cap;
    return a;
}

bool misaligned(const void* ptr, uintptr_t a) { return (reinterpret_cast<uintptr_t>(ptr) & (a - 1)) != 0; }

// Shared checks of lc_batch_compress / lc_batch_sizes.
lc_status check_batch_fit(const void* d_keys, const lc_batch_list* d_lists, const lc_batch_params* p, void* d_ws,
                          uint64_t ws_bytes, uint64_t* d_sizes, uint32_t* d_stats, lc::Workspace* W)
{
    lc_status st = check_batch(p);
    if (st != LC_OK) return st;
    if (p->total_blocks > (kMaxKeys >> p->log2_block) * p->nlists || p->total_groups > p->total_blocks)
        return LC_EINVAL;
    if (!d_lists || !d_stats || misaligned(d_lists, 8) || misaligned(d_stats, 4) ||
        (d_sizes && misaligned(d_sizes, 8)))
        return LC_EINVAL;
    if (p->total_blocks && (!d_keys || !d_ws || misaligned(d_keys, p->key_bytes) || misaligned(d_ws, 16)))
        return LC_EINVAL;
    const BatchWs w = plan_batch_ws(p->total_blocks, p->log2_block, p->fit);
    if (p->total_blocks && ws_bytes < w.total) return LC_ENOSPC;
    uint8_t* ws = static_cast<uint8_t*>(d_ws);
    *W = lc::Workspace{};
    if (p->total_blocks) {
        W->blk = reinterpret_cast<lc::BlockInfo*>(ws + w.blk);
        W->seg_start = reinterpret_cast<uint16_t*>(ws + w.start);
        W->seg_delta = reinterpret_cast<uint64_t*>(ws + w.delta);
        W->seg_A = reinterpret_cast<uint64_t*>(ws + w.slope);
        W->seg_frac = p->fit == LC_FIT_OPT ? reinterpret_cast<uint32_t*>(ws + w.frac) : nullptr;
    }
    return LC_OK;
}

}  // namespace

lc_status lc::layout_from_info(const lc_blob_info* info, lc::Layout* L) { return layout_of(info, L); }

LC_API lc_status lc_compress_bound(uint64_t n, const lc_params* p, uint64_t* blob_max, uint64_t* ws_bytes)
{
    lc_status st = check_params(p);
    if (st != LC_OK) return st;
    if (n > kMaxKeys) return LC_EINVAL;
    const lc::Layout L = fixed_layout(n, p);
    if (blob_max) *blob_max = worst_blob(L);
    if (ws_bytes) *ws_bytes = plan_workspace(L).total;
    return LC_OK;
}

LC_API lc_status lc_compress(const void* d_keys, uint64_t n, const lc_params* p, void* d_blob, uint64_t blob_cap,
                             void* d_ws, uint64_t ws_bytes, uint64_t* d_blob_bytes, uint32_t* d_flags,
                             void* stream)
{
    lc_status st = check_params(p);
    if (st != LC_OK) return st;
    if (n > kMaxKeys || !d_blob || !d_flags || (n && (!d_keys || !d_ws))) return LC_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_blob) & 15) || (reinterpret_cast<uintptr_t>(d_ws) & 15) ||
        (reinterpret_cast<uintptr_t>(d_keys) & (p->key_bytes - 1)))
        return LC_EINVAL;
    const lc::Layout L = fixed_layout(n, p);
    const WsPlan w = plan_workspace(L);
    if (blob_cap < worst_blob(L)) return LC_ENOSPC;
    if (n && ws_bytes < w.total) return LC_ENOSPC;
    uint8_t* ws = static_cast<uint8_t*>(d_ws);
    lc::Workspace W{};
    if (n) {
        W.blk = reinterpret_cast<lc::BlockInfo*>(ws + w.blk);
        W.tiles = reinterpret_cast<lc::TileSum*>(ws + w.tiles);
        W.seg_start = reinterpret_cast<uint16_t*>(ws + w.start);
        W.seg_delta = reinterpret_cast<uint64_t*>(ws + w.delta);
        W.seg_A = reinterpret_cast<uint64_t*>(ws + w.slope);
        W.seg_frac = L.flags ? reinterpret_cast<uint32_t*>(ws + w.frac) : nullptr;
    }
    hipError_t e = lc::launch_compress(d_keys, L, p->fit, static_cast<uint8_t*>(d_blob), W, d_blob_bytes, d_flags,
                                       static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LC_OK : LC_EDEVICE;
}

LC_API lc_status lc_info(const void* h_header, uint64_t header_bytes, lc_blob_info* out)
{
    if (!h_header || !out) return LC_EINVAL;
    if (header_bytes < LC_HEADER_BYTES) return LC_EFORMAT;
    const uint8_t* h = static_cast<const uint8_t*>(h_header);
    if (rd(h, 4) != kMagic || rd(h + 4, 2) != 1) return LC_EFORMAT;
    lc_blob_info I{};
    I.key_bytes = h[6];
    I.log2_block = h[7];
    I.frac_bits = h[8];
    I.width = h[9];
    I.flags = h[10];
    if (h[11] != 0) return LC_EFORMAT;
    I.eps = (uint32_t)rd(h + 12, 4);
    I.n = rd(h + 16, 8);
    I.nblocks = rd(h + 24, 8);
    I.nseg_total = rd(h + 32, 8);
    I.max_nseg = (uint32_t)rd(h + 40, 4);
    I.max_seg_bytes = (uint32_t)rd(h + 44, 4);
    I.off_first = rd(h + 48, 8);
    I.off_dir = rd(h + 56, 8);
    I.off_res = rd(h + 64, 8);
    I.res_stride = rd(h + 72, 8);
    I.off_seg = rd(h + 80, 8);
    I.blob_bytes = rd(h + 88, 8);
    lc::Layout L;
    if (layout_of(&I, &L) != LC_OK) return LC_EFORMAT;
    if (I.blob_bytes < I.off_seg || I.nseg_total < I.nblocks || I.nseg_total > I.n) return LC_EFORMAT;
    *out = I;
    return LC_OK;
}

LC_API lc_status lc_decompress(const void* d_blob, const lc_blob_info* info, void* d_out, void* stream)
{
    lc::Layout L;
    if (!d_blob || layout_of(info, &L) != LC_OK) return LC_EINVAL;
    if (L.n == 0) return LC_OK;
    if (!d_out || (reinterpret_cast<uintptr_t>(d_out) & (L.kb - 1))) return LC_EINVAL;
    hipError_t e = lc::launch_decode(static_cast<const uint8_t*>(d_blob), L, 0, L.n, d_out,
                                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LC_OK : LC_EDEVICE;
}

LC_API lc_status lc_decompress_range(const void* d_blob, const lc_blob_info* info, uint64_t begin, uint64_t end,
                                     void* d_out, void* stream)
{
    lc::Layout L;
    if (!d_blob || layout_of(info, &L) != LC_OK) return LC_EINVAL;
    if (begin > end || end > L.n) return LC_EINVAL;
    if (begin == end) return LC_OK;
    if (!d_out || (reinterpret_cast<uintptr_t>(d_out) & (L.kb - 1))) return LC_EINVAL;
    hipError_t e = lc::launch_decode(static_cast<const uint8_t*>(d_blob), L, begin, end, d_out,
                                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LC_OK : LC_EDEVICE;
}

LC_API lc_status lc_access(const void* d_blob, const lc_blob_info* info, const uint64_t* d_idx, uint64_t m,
                           void* d_out, uint32_t* d_flags, void* stream)
{
    lc::Layout L;
    if (!d_blob || layout_of(info, &L) != LC_OK) return LC_EINVAL;
    if (m == 0) return LC_OK;
    if (!d_idx || !d_out || !d_flags || (reinterpret_cast<uintptr_t>(d_out) & (L.kb - 1)) ||
        (reinterpret_cast<uintptr_t>(d_idx) & 7))
        return LC_EINVAL;
    hipError_t e = lc::launch_access(static_cast<const uint8_t*>(d_blob), L, d_idx, m, d_out, d_flags,
                                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LC_OK : LC_EDEVICE;
}

LC_API lc_status lc_lower_bound(const void* d_blob, const lc_blob_info* info, const void* d_q, uint64_t m,
                                uint64_t* d_pos, void* stream)
{
    lc::Layout L;
    if (!d_blob || layout_of(info, &L) != LC_OK) return LC_EINVAL;
    if (m == 0) return LC_OK;
    if (!d_q || !d_pos || (reinterpret_cast<uintptr_t>(d_q) & (L.kb - 1)) ||
        (reinterpret_cast<uintptr_t>(d_pos) & 7))
        return LC_EINVAL;
    hipError_t e = lc::launch_lower_bound(static_cast<const uint8_t*>(d_blob), L, d_q, m, d_pos,
                                          static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LC_OK : LC_EDEVICE;
}

LC_API lc_status lc_quantile(const void* d_blob, const lc_blob_info* info, const uint64_t* d_k, uint64_t q,
                             uint64_t m, uint32_t approx, void* d_out, void* stream)
{
    lc::Layout L;
    if (!d_blob || layout_of(info, &L) != LC_OK || L.n == 0 || q == 0) return LC_EINVAL;
    if (m == 0) return LC_OK;
    if (!d_k || !d_out || (reinterpret_cast<uintptr_t>(d_k) & 7) || (reinterpret_cast<uintptr_t>(d_out) & (L.kb - 1)))
        return LC_EINVAL;
    hipError_t e = lc::launch_quantile(static_cast<const uint8_t*>(d_blob), L, d_k, q, m, approx != 0, d_out,
                                       static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LC_OK : LC_EDEVICE;
}

LC_API lc_status lc_decompress_approx(const void* d_blob, const lc_blob_info* info, uint64_t begin, uint64_t end,
                                      void* d_out, void* stream)
{
    lc::Layout L;
    if (!d_blob || layout_of(info, &L) != LC_OK) return LC_EINVAL;
    if (begin > end || end > L.n) return LC_EINVAL;
    if (begin == end) return LC_OK;
    if (!d_out || (reinterpret_cast<uintptr_t>(d_out) & (L.kb - 1))) return LC_EINVAL;
    hipError_t e = lc::launch_decode(static_cast<const uint8_t*>(d_blob), L, begin, end, d_out,
                                     static_cast<hipStream_t>(stream), true);
    return e == hipSuccess ? LC_OK : LC_EDEVICE;
}

namespace {

struct SetPlan {
    uint64_t a_keys, b_keys, fa, fb, PA, PB, cnt, tot, total;
};

// probe: the decoded side of an AND (the smaller list)
SetPlan plan_setop(uint32_t op, uint64_t na, uint64_t nb, uint32_t kb)
{
    const uint64_t T = lc::kSetTileKeys;
    const uint64_t ta = (na + T - 1) / T, tb = op == LC_SETOP_UNION ? (nb + T - 1) / T : 0;
    const bool u = op == LC_SETOP_UNION;
    SetPlan p;
    p.a_keys = 0;
    p.b_keys = p.a_keys + lc::align16(na * kb);
    p.fa = p.b_keys + (u ? lc::align16(nb * kb) : 0);
    p.fb = p.fa + lc::align16(na);
    p.PA = p.fb + (u ? lc::align16(nb) : 0);
    p.PB = p.PA + (u ? lc::align16((na + 1) * 8) : 0);
    p.cnt = p.PB + (u ? lc::align16((nb + 1) * 8) : 0);
    p.tot = p.cnt + lc::align16((ta + tb + 2) * 8);
    p.total = p.tot + 16;
    return p;
}

lc_status check_setop(const lc_blob_info* a, const lc_blob_info* b, uint32_t op, lc::Layout* La, lc::Layout* Lb)
{
    if (op != LC_SETOP_INTERSECT && op != LC_SETOP_UNION) return LC_EINVAL;
    if (layout_of(a, La) != LC_OK || layout_of(b, Lb) != LC_OK || La->kb != Lb->kb) return LC_EINVAL;
    return LC_OK;
}

}  // namespace

LC_API lc_status lc_setop_bound(const lc_blob_info* a, const lc_blob_info* b, uint32_t op, uint64_t* out_max,
                                uint64_t* ws_bytes)
{
    lc::Layout La, Lb;
    lc_status st = check_setop(a, b, op, &La, &Lb);
    if (st != LC_OK) return st;
    const bool swap = op == LC_SETOP_INTERSECT && La.n > Lb.n;
    const uint64_t na = swap ? Lb.n : La.n, nb = swap ? La.n : Lb.n;
    if (out_max) *out_max = op == LC_SETOP_INTERSECT ? na : na + nb;
    if (ws_bytes) *ws_bytes = plan_setop(op, na, nb, La.kb).total;
    return LC_OK;
}

LC_API lc_status lc_setop(uint32_t op, const void* d_blob_a, const lc_blob_info* a, const void* d_blob_b,
                          const lc_blob_info* b, void* d_ws, uint64_t ws_bytes, void* d_out, uint64_t out_cap,
                          uint64_t* d_count, void* stream)
{
    lc::Layout La, Lb;
    lc_status st = check_setop(a, b, op, &La, &Lb);
    if (st != LC_OK) return st;
    if (!d_blob_a || !d_blob_b || !d_ws || !d_count || (reinterpret_cast<uintptr_t>(d_ws) & 15) ||
        (reinterpret_cast<uintptr_t>(d_count) & 7))
        return LC_EINVAL;
    // AND probes the larger list with the keys of the smaller one
    const bool swap = op == LC_SETOP_INTERSECT && La.n > Lb.n;
    const uint8_t* pa = static_cast<const uint8_t*>(swap ? d_blob_b : d_blob_a);
    const uint8_t* pb = static_cast<const uint8_t*>(swap ? d_blob_a : d_blob_b);
    if (swap) std::swap(La, Lb);
    const uint64_t need = op == LC_SETOP_INTERSECT ? La.n : La.n + Lb.n;
    if (out_cap < need) return LC_ENOSPC;
    if (need && (!d_out || (reinterpret_cast<uintptr_t>(d_out) & (La.kb - 1)))) return LC_EINVAL;
    const SetPlan p = plan_setop(op, La.n, Lb.n, La.kb);
    if (ws_bytes < p.total) return LC_ENOSPC;
    uint8_t* ws = static_cast<uint8_t*>(d_ws);
    lc::SetWs w;
    w.a_keys = ws + p.a_keys;
    w.b_keys = ws + p.b_keys;
    w.fa = ws + p.fa;
    w.fb = ws + p.fb;
    w.PA = reinterpret_cast<uint64_t*>(ws + p.PA);
    w.PB = reinterpret_cast<uint64_t*>(ws + p.PB);
    w.cnt = reinterpret_cast<uint64_t*>(ws + p.cnt);
    w.tot = reinterpret_cast<uint64_t*>(ws + p.tot);
    hipError_t e = lc::launch_setop(op, pa, La, pb, Lb, w, d_out, d_count, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LC_OK : LC_EDEVICE;
}

LC_API lc_status lc_batch_plan(lc_batch_params* p, lc_batch_list* h_lists)
{
    lc_status st = check_batch(p);
    if (st != LC_OK) return st;
    if (!h_lists) return LC_EINVAL;
    lc_params q{};
    q.key_bytes = p->key_bytes;
    q.log2_block = p->log2_block;
    q.frac_bits = p->frac_bits;
    q.fit = (uint8_t)p->fit;
    q.eps = p->max_eps;
    uint64_t blob = 0, blocks = 0, groups = 0;
    for (uint32_t l = 0; l < p->nlists; l++) {
        lc_batch_list& li = h_lists[l];
        if (li.n > kMaxKeys) return LC_EINVAL;
        const lc::Layout L = fixed_layout(li.n, &q);
        const uint64_t cap = worst_blob(L);
        li.blob_off = blob;
        li.blob_cap = cap;
        li.block_off = blocks;
        li.group_off = groups;
        blob += cap;
        blocks += L.nblocks;
        groups += (L.nblocks + 3) / 4;
        if (blob >> 62) return LC_EINVAL;
    }
    p->total_blocks = blocks;
    p->total_groups = groups;
    p->blob_bytes = blob;
    p->ws_bytes = plan_batch_ws(blocks, p->log2_block, p->fit).total;
    return LC_OK;
}

LC_API lc_status lc_batch_compress(const void* d_keys, uint64_t nkeys, const lc_batch_list* d_lists,
                                   const lc_batch_params* p, void* d_blob, uint64_t blob_cap, void* d_ws,
                                   uint64_t ws_bytes, uint64_t* d_sizes, uint32_t* d_stats, void* stream)
{
    lc::Workspace W;
    lc_status st = check_batch_fit(d_keys, d_lists, p, d_ws, ws_bytes, d_sizes, d_stats, &W);
    if (st != LC_OK) return st;
    if (!d_blob || misaligned(d_blob, 16)) return LC_EINVAL;
    if (blob_cap < p->blob_bytes) return LC_ENOSPC;
    const lc::BatchArgs a = batch_args(p, nkeys, blob_cap);
    hipError_t e = lc::launch_batch_compress(d_keys, d_lists, a, nullptr, 0, static_cast<uint8_t*>(d_blob), W, d_sizes,
                                             d_stats, false, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LC_OK : LC_EDEVICE;
}

static lc_status check_cands(const lc_batch_params* p, const uint32_t* h_cands, uint32_t ncand)
{
    if (!h_cands || ncand == 0 || ncand > LC_BATCH_MAX_CANDIDATES) return LC_EINVAL;
    for (uint32_t k = 0; k < ncand; k++) {
        if (h_cands[k] > p->max_eps) return LC_EINVAL;
        if (k && h_cands[k] <= h_cands[k - 1]) return LC_EINVAL;
    }
    return LC_OK;
}

LC_API lc_status lc_batch_sizes(const void* d_keys, uint64_t nkeys, const lc_batch_list* d_lists,
                                const lc_batch_params* p, const uint32_t* h_cands, uint32_t ncand, void* d_ws,
                                uint64_t ws_bytes, uint64_t* d_sizes, uint32_t* d_stats, void* stream)
{
    lc::Workspace W;
    lc_status st = check_batch_fit(d_keys, d_lists, p, d_ws, ws_bytes, d_sizes, d_stats, &W);
    if (st != LC_OK) return st;
    if (!d_sizes || (st = check_cands(p, h_cands, ncand)) != LC_OK) return LC_EINVAL;
    const lc::BatchArgs a = batch_args(p, nkeys, ~0ull);
    hipError_t e = lc::launch_batch_compress(d_keys, d_lists, a, h_cands, ncand, nullptr, W, d_sizes, d_stats, true,
                                             static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LC_OK : LC_EDEVICE;
}

LC_API lc_status lc_batch_pick_eps(lc_batch_list* d_lists, const lc_batch_params* p, const uint64_t* d_sizes,
                                   const uint32_t* h_cands, uint32_t ncand, void* stream)
{
    lc_status st = check_batch(p);
    if (st != LC_OK) return st;
    if (!d_lists || !d_sizes || misaligned(d_lists, 8) || misaligned(d_sizes, 8)) return LC_EINVAL;
    if ((st = check_cands(p, h_cands, ncand)) != LC_OK) return st;
    hipError_t e = lc::launch_batch_pick(d_lists, p->nlists, d_sizes, h_cands, ncand, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LC_OK : LC_EDEVICE;
}

LC_API lc_status lc_batch_decompress(const void* d_blob, uint64_t blob_cap, const lc_batch_list* d_lists,
                                     const lc_batch_params* p, uint32_t max_seg_bytes, void* d_out, uint64_t nout,
                                     uint32_t* d_stats, void* stream)
{
    lc_status st = check_batch(p);
    if (st != LC_OK) return st;
    if (p->total_blocks > (kMaxKeys >> p->log2_block) * p->nlists || p->total_groups > p->total_blocks)
        return LC_EINVAL;
    if (!d_lists || !d_stats || misaligned(d_lists, 8) || misaligned(d_stats, 4)) return LC_EINVAL;
    if (p->total_blocks == 0) return LC_OK;
    if (!d_blob || !d_out || misaligned(d_blob, 16) || misaligned(d_out, p->key_bytes)) return LC_EINVAL;
    const lc::BatchArgs a = batch_args(p, nout, blob_cap);
    hipError_t e = lc::launch_batch_decode(static_cast<const uint8_t*>(d_blob), d_lists, a, max_seg_bytes, d_out,
                                           d_stats, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LC_OK : LC_EDEVICE;
}

namespace {

struct PairPlan {
    uint64_t keys, flags, cnt, tot, P, total;
};

PairPlan plan_pairs(uint64_t total_keys, uint32_t kb)
{
    const uint64_t tiles = (total_keys + lc::kSetTileKeys - 1) / lc::kSetTileKeys;
    PairPlan p;
    p.keys = 0;
    p.flags = lc::align16(total_keys * kb);
    p.cnt = p.flags + lc::align16(total_keys);
    p.tot = p.cnt + lc::align16((tiles + 2) * 8);
    p.P = p.tot + 16;
    p.total = p.P + lc::align16((total_keys + 1) * 8);
    return p;
}

}  // namespace

LC_API lc_status lc_batch_and_plan(const lc_batch_params* p, const lc_batch_list* h_lists, lc_list_pair* h_pairs,
                                   uint32_t npairs, uint64_t* total_keys, uint64_t* total_blocks, uint64_t* ws_bytes)
{
    lc_status st = check_batch(p);
    if (st != LC_OK) return st;
    if (!h_lists || (npairs && !h_pairs)) return LC_EINVAL;
    const uint64_t B = 1ull << p->log2_block;
    uint64_t keys = 0, blocks = 0;
    for (uint32_t i = 0; i < npairs; i++) {
        lc_list_pair& pr = h_pairs[i];
        if (pr.a >= p->nlists || pr.b >= p->nlists) return LC_EINVAL;
        const bool a_probe = h_lists[pr.a].n <= h_lists[pr.b].n;
        pr.probe = a_probe ? pr.a : pr.b;
        pr.target = a_probe ? pr.b : pr.a;
        pr.n = h_lists[pr.probe].n;
        if (pr.n > kMaxKeys) return LC_EINVAL;
        pr.key_off = keys;
        pr.block_off = blocks;
        keys += pr.n;
        blocks += (pr.n + B - 1) / B;
        if (keys >> 50) return LC_EINVAL;
    }
    if (total_keys) *total_keys = keys;
    if (total_blocks) *total_blocks = blocks;
    if (ws_bytes) *ws_bytes = plan_pairs(keys, p->key_bytes).total;
    return LC_OK;
}

LC_API lc_status lc_batch_and(const void* d_blob, uint64_t blob_cap, const lc_batch_list* d_lists,
                              const lc_batch_params* p, const lc_list_pair* d_pairs, uint32_t npairs,
                              uint64_t total_keys, uint64_t total_blocks, uint32_t max_seg_bytes, void* d_ws,
                              uint64_t ws_bytes, void* d_out, uint64_t* d_counts, uint32_t* d_stats, void* stream)
{
    lc_status st = check_batch(p);
    if (st != LC_OK) return st;
    if (npairs == 0) return LC_OK;
    if (!d_blob || !d_lists || !d_pairs || !d_ws || !d_counts || !d_stats || misaligned(d_blob, 16) ||
        misaligned(d_lists, 8) || misaligned(d_pairs, 8) || misaligned(d_ws, 16) || misaligned(d_counts, 8) ||
        misaligned(d_stats, 4))
        return LC_EINVAL;
    if (total_keys > kMaxKeys || total_blocks > total_keys) return LC_EINVAL;
    if (total_keys && (!d_out || misaligned(d_out, p->key_bytes))) return LC_EINVAL;
    const PairPlan pl = plan_pairs(total_keys, p->key_bytes);
    if (ws_bytes < pl.total) return LC_ENOSPC;
    uint8_t* ws = static_cast<uint8_t*>(d_ws);
    lc::PairWs w;
    w.keys = ws + pl.keys;
    w.flags = ws + pl.flags;
    w.cnt = reinterpret_cast<uint64_t*>(ws + pl.cnt);
    w.tot = reinterpret_cast<uint64_t*>(ws + pl.tot);
    w.P = reinterpret_cast<uint64_t*>(ws + pl.P);
    lc::BatchArgs a = batch_args(p, ~0ull, blob_cap);  // key offsets of the table are not used here
    hipError_t e = lc::launch_batch_and(static_cast<const uint8_t*>(d_blob), d_lists, a, d_pairs, npairs, total_keys,
                                        total_blocks, max_seg_bytes, w, d_out, d_counts, d_stats,
                                        static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LC_OK : LC_EDEVICE;
}

LC_API const char* lc_strerror(lc_status s)
{
    switch (s) {
    case LC_OK: return "ok";
    case LC_EINVAL: return "invalid argument";
    case LC_ENOSPC: return "buffer too small";
    case LC_EFORMAT: return "not a valid blob header";
    case LC_EDEVICE: return "kernel launch failed";
    case LC_ETOOBIG: return "input too large for the static scratch of lc_compress_noalloc";
    default: return "unknown status";
    }
}
