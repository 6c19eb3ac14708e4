// Output arena of the request server: a ring over a fixed byte range that
// hands out 16-byte aligned regions in admission order and takes them back
// in any order.  Host-only and free of HIP, so it is unit-tested on the CPU.
//
// Live regions always form one contiguous run of the ring, oldest first,
// possibly wrapping once past the end of the range.  A region freed out of
// order stays reserved until every older region is freed too; then the
// run's tail jumps past all of them.  An allocation that does not fit before
// the end of the range wraps to offset 0, leaving the end of the range
// unused until the run drains past it.
#pragma once

#include <stdint.h>

#include <deque>
#include <unordered_map>

namespace lc {

class Arena {
public:
    static constexpr uint64_t kNone = ~uint64_t(0);

    explicit Arena(uint64_t bytes) : size_(bytes & ~uint64_t(15)) {}

    uint64_t size() const { return size_; }
    uint64_t live_bytes() const { return live_; }
    size_t live_regions() const { return by_off_.size(); }

    // Offset of a new region of `bytes` (rounded up to a multiple of 16, at
    // least 16), or kNone when it does not fit now.  A region larger than
    // the arena never fits.
    uint64_t alloc(uint64_t bytes)
    {
        const uint64_t x = bytes <= 16 ? 16 : (bytes + 15) & ~uint64_t(15);
        if (x > size_ || bytes > size_) return kNone;
        if (regions_.empty()) {
            head_ = tail_ = 0;
            wrapped_ = false;
        }
        uint64_t off;
        if (!wrapped_) {  // free: [head, size) and [0, tail)
            if (size_ - head_ >= x) {
                off = head_;
            } else if (tail_ >= x) {
                off = 0;
                wrapped_ = true;
            } else {
                return kNone;
            }
        } else {  // free: [head, tail)
            if (tail_ - head_ < x) return kNone;
            off = head_;
        }
        head_ = off + x;
        regions_.push_back(Region{off, x, false});
        by_off_[off] = front_seq_ + regions_.size() - 1;
        live_ += x;
        return off;
    }

    // Gives back the region at `off`; false if no live region starts there.
    bool free(uint64_t off)
    {
        auto it = by_off_.find(off);
        if (it == by_off_.end()) return false;
        Region& r = regions_[it->second - front_seq_];
        by_off_.erase(it);
        r.freed = true;
        live_ -= r.bytes;
        while (!regions_.empty() && regions_.front().freed) {
            regions_.pop_front();
            front_seq_++;
            if (!regions_.empty()) {
                if (regions_.front().off < tail_) wrapped_ = false;  // drained past the wrap point
                tail_ = regions_.front().off;
            }
        }
        if (regions_.empty()) {
            head_ = tail_ = 0;
            wrapped_ = false;
        }
        return true;
    }

private:
    struct Region {
        uint64_t off, bytes;
        bool freed;
    };
    uint64_t size_;
    uint64_t head_ = 0, tail_ = 0;  // next free byte; start of the oldest live region
    bool wrapped_ = false;          // the live run crosses the end of the range
    uint64_t live_ = 0;
    uint64_t front_seq_ = 0;        // sequence number of regions_.front()
    std::deque<Region> regions_;    // live (and freed-but-younger-than-live) regions, oldest first
    std::unordered_map<uint64_t, uint64_t> by_off_;  // live region offset -> sequence number
};

}  // namespace lc
