// Request server over one device-resident blob (declared in include/lc.h):
// admission by the output arena, continuous batching into launches of the
// serve kernel, up to max_inflight launches in flight on their own streams.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <new>
#include <numeric>
#include <vector>

#include "lc.h"
#include "lc_arena.h"
#include "lc_launch.h"

#define LC_API extern "C" __attribute__((visibility("default")))

namespace {

using Clock = std::chrono::steady_clock;
constexpr uint64_t kMaxItems = 1ull << 22;  // range blocks per launch (a lone request may exceed it)

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    lc::ServeRange* d_ranges = nullptr;  // max_batch entries (device)
    lc::ServePoint* d_points = nullptr;  // max_batch entries (device)
    lc::ServeRange* h_ranges = nullptr;  // pinned staging of the same
    lc::ServePoint* h_points = nullptr;
    std::vector<uint64_t> reqs;          // requests of the launch in flight
    bool busy = false;
};

}  // namespace

struct lc_server {
    const uint8_t* blob = nullptr;
    lc::Layout L{};
    uint8_t* arena_base = nullptr;
    lc::Arena arena{0};
    uint32_t max_batch = 0, max_inflight = 0;
    int device = 0;
    std::vector<Slot> slots;
};

namespace {

void release(lc_server* s)
{
    for (Slot& sl : s->slots) {
        // teardown: nothing to report a failure to
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.d_ranges) (void)hipFree(sl.d_ranges);
        if (sl.d_points) (void)hipFree(sl.d_points);
        if (sl.h_ranges) (void)hipHostFree(sl.h_ranges);
        if (sl.h_points) (void)hipHostFree(sl.h_points);
    }
    delete s;
}

uint64_t out_bytes(const lc_request& r, uint32_t kb)
{
    switch (r.op) {
    case LC_OP_RANGE: return (r.b - r.a) * kb;
    case LC_OP_ACCESS: return kb;
    default: return 8;
    }
}

}  // namespace

LC_API lc_status lc_server_create(const void* d_blob, const lc_blob_info* info, void* d_arena, uint64_t arena_bytes,
                                  const lc_serve_config* cfg, lc_server** out)
{
    if (!out) return LC_EINVAL;
    *out = nullptr;
    lc::Layout L;
    if (!d_blob || !d_arena || !cfg || lc::layout_from_info(info, &L) != LC_OK) return LC_EINVAL;
    if (arena_bytes < 16 || (reinterpret_cast<uintptr_t>(d_arena) & 15) || (reinterpret_cast<uintptr_t>(d_blob) & 15))
        return LC_EINVAL;
    if (cfg->max_batch < 1 || cfg->max_batch > 65536 || cfg->max_inflight < 1 || cfg->max_inflight > 16)
        return LC_EINVAL;
    lc_server* s = new (std::nothrow) lc_server();
    if (!s) return LC_EDEVICE;
    s->blob = static_cast<const uint8_t*>(d_blob);
    s->L = L;
    s->arena_base = static_cast<uint8_t*>(d_arena);
    s->arena = lc::Arena(arena_bytes);
    s->max_batch = cfg->max_batch;
    s->max_inflight = cfg->max_inflight;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return LC_EDEVICE;
    }
    s->slots.resize(cfg->max_inflight);
    for (Slot& sl : s->slots) {
        const size_t rb = sizeof(lc::ServeRange) * cfg->max_batch, pb = sizeof(lc::ServePoint) * cfg->max_batch;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipMalloc(&sl.d_ranges, rb) != hipSuccess || hipMalloc(&sl.d_points, pb) != hipSuccess ||
            hipHostMalloc(&sl.h_ranges, rb, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&sl.h_points, pb, hipHostMallocDefault) != hipSuccess) {
            release(s);
            return LC_EDEVICE;
        }
        sl.reqs.reserve(cfg->max_batch);
    }
    *out = s;
    return LC_OK;
}

LC_API lc_status lc_server_destroy(lc_server* s)
{
    if (!s) return LC_EINVAL;
    release(s);
    return LC_OK;
}

LC_API lc_status lc_server_run(lc_server* s, const lc_request* reqs, uint64_t n, lc_request_result* res,
                               lc_serve_stats* stats)
{
    if (!s || (n && (!reqs || !res))) return LC_EINVAL;
    if (hipSetDevice(s->device) != hipSuccess) return LC_EDEVICE;
    const uint32_t kb = s->L.kb;
    lc_serve_stats st{};
    std::vector<uint64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint64_t x, uint64_t y) { return reqs[x].arrival_ns < reqs[y].arrival_ns; });
    std::vector<uint64_t> off(n, lc::Arena::kNone);
    for (uint64_t i = 0; i < n; i++) res[i] = lc_request_result{-1, -1, -1, LC_OK, 0};

    const Clock::time_point t0 = Clock::now();
    auto now = [&]() { return (int64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count(); };
    uint64_t next = 0, done = 0;
    std::deque<uint64_t> queue;
    lc_status rc = LC_OK;
    auto finish = [&](uint64_t r, int32_t status, int64_t t) {
        res[r].status = status;
        if (res[r].admit_ns < 0) res[r].admit_ns = t;
        if (res[r].launch_ns < 0) res[r].launch_ns = t;
        res[r].complete_ns = t;
        done++;
    };

    while (done < n) {
        // arrivals
        int64_t t = now();
        while (next < n && (int64_t)reqs[order[next]].arrival_ns <= t) queue.push_back(order[next++]);
        // completions
        for (Slot& sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            const int64_t tc = now();
            for (uint64_t r : sl.reqs) {
                s->arena.free(off[r]);
                finish(r, q == hipSuccess ? LC_OK : LC_EDEVICE, tc);
            }
            if (q != hipSuccess) rc = LC_EDEVICE;
            sl.reqs.clear();
            sl.busy = false;
        }
        if (rc != LC_OK) break;
        // admission into a free slot
        Slot* sl = nullptr;
        for (Slot& x : s->slots)
            if (!x.busy) {
                sl = &x;
                break;
            }
        if (!sl || queue.empty()) continue;
        t = now();
        uint32_t nr = 0, np = 0;
        uint64_t items = 0;
        while (!queue.empty() && nr + np < s->max_batch) {
            const uint64_t r = queue.front();
            const lc_request& q = reqs[r];
            const bool ok = (q.op == LC_OP_RANGE && q.a <= q.b && q.b <= s->L.n) ||
                            (q.op == LC_OP_ACCESS && q.a < s->L.n) || q.op == LC_OP_LOWER_BOUND;
            if (!ok) {
                queue.pop_front();
                finish(r, LC_EINVAL, t);
                continue;
            }
            if (q.op == LC_OP_RANGE && q.a == q.b) {  // nothing to decode
                queue.pop_front();
                finish(r, LC_OK, t);
                continue;
            }
            const uint64_t nb = q.op == LC_OP_RANGE ? ((q.b - 1) >> s->L.log2b) - (q.a >> s->L.log2b) + 1 : 0;
            if (items && items + nb > kMaxItems) break;  // the launch is full
            const uint64_t bytes = out_bytes(q, kb);
            if (bytes > s->arena.size()) {
                queue.pop_front();
                finish(r, LC_ENOSPC, t);
                continue;
            }
            const uint64_t o = s->arena.alloc(bytes);
            if (o == lc::Arena::kNone) {  // wait for completions to free space (arrival order is kept)
                st.arena_waits++;
                break;
            }
            queue.pop_front();
            off[r] = o;
            res[r].admit_ns = t;
            if (q.op == LC_OP_RANGE) {
                sl->h_ranges[nr++] = lc::ServeRange{q.a, q.b, o, items};
                items += nb;
            } else {
                lc::ServePoint p{};
                p.key = q.a;
                p.out_off = o;
                p.op = q.op;
                sl->h_points[np++] = p;
            }
            sl->reqs.push_back(r);
        }
        st.peak_arena_bytes = std::max<uint64_t>(st.peak_arena_bytes, s->arena.live_bytes());
        if (sl->reqs.empty()) continue;
        lc::ServeArgs a{};
        a.L = s->L;
        a.nrange = nr;
        a.npoint = np;
        a.range_items = items;
        hipError_t e = hipSuccess;
        if (nr) e = hipMemcpyAsync(sl->d_ranges, sl->h_ranges, sizeof(lc::ServeRange) * nr, hipMemcpyHostToDevice,
                                   sl->stream);
        if (e == hipSuccess && np)
            e = hipMemcpyAsync(sl->d_points, sl->h_points, sizeof(lc::ServePoint) * np, hipMemcpyHostToDevice,
                               sl->stream);
        if (e == hipSuccess) e = lc::launch_serve(s->blob, a, sl->d_ranges, sl->d_points, s->arena_base, sl->stream);
        for (uint64_t r : sl->reqs) {
            if (e != hipSuccess) break;
            if (reqs[r].d_dest)
                e = hipMemcpyAsync(reqs[r].d_dest, s->arena_base + off[r], out_bytes(reqs[r], kb),
                                   hipMemcpyDeviceToDevice, sl->stream);
        }
        if (e == hipSuccess) e = hipEventRecord(sl->done, sl->stream);
        const int64_t tl = now();
        for (uint64_t r : sl->reqs) {
            res[r].launch_ns = tl;
            res[r].launch = (uint32_t)st.launches;
        }
        st.launches++;
        st.max_batch_seen = std::max<uint64_t>(st.max_batch_seen, sl->reqs.size());
        sl->busy = true;
        if (e != hipSuccess) {
            rc = LC_EDEVICE;
            break;
        }
    }
    if (rc != LC_OK) {
        // drain what is in flight, then fail everything unfinished
        for (Slot& sl : s->slots) {
            if (!sl.busy) continue;
            (void)hipStreamSynchronize(sl.stream);  // already failing: only waits
            for (uint64_t r : sl.reqs) s->arena.free(off[r]);
            sl.reqs.clear();
            sl.busy = false;
        }
        const int64_t t = now();
        for (uint64_t i = 0; i < n; i++)
            if (res[i].complete_ns < 0) finish(i, LC_EDEVICE, t);
    }
    if (stats) *stats = st;
    return rc;
}
