// gfq_sched.h -- host-side scheduling core of the product server: a device-memory arena
// bounded by a byte budget, and the admission queue ordered by arrival.  Plain C++ with no
// HIP calls (device memory is obtained through callbacks), so the same code runs in the
// library and in host-only checks.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <functional>
#include <map>
#include <queue>
#include <vector>

namespace gfq {

// Offsets handed out from chunks of device memory.  Every chunk comes from `grow` and the
// sum of chunk sizes never exceeds `budget`; allocation is first fit over a free list per
// chunk with neighbours coalesced on release.  A chunk is returned through `shrink` only by
// reset(), which the caller uses when nothing is allocated (so a request larger than every
// free extent can still be placed once the device is idle).
class Arena {
  public:
    typedef std::function<bool(size_t, uintptr_t *)> GrowFn;
    typedef std::function<void(uintptr_t)> ShrinkFn;
    static constexpr size_t kAlign = 256;

    Arena(size_t budget, size_t chunk, GrowFn grow, ShrinkFn shrink)
        : budget_(budget), chunk_(std::max(chunk, kAlign)), grow_(grow), shrink_(shrink) {}
    ~Arena() { reset(); }

    static size_t round(size_t b) { return (std::max<size_t>(b, 1) + kAlign - 1) & ~(kAlign - 1); }

    // Reserve `bytes` (rounded up to 256); false when it does not fit now.
    bool alloc(size_t bytes, uintptr_t *out) {
        const size_t need = round(bytes);
        if (need > budget_) return false;
        for (Chunk &c : chunks_)
            if (take(c, need, out)) return true;
        const size_t room = budget_ - held_;
        if (need > room) return false;
        const size_t size = std::min(room, std::max(need, chunk_));
        uintptr_t base = 0;
        if (!grow_(size, &base)) return false;
        chunks_.push_back(Chunk{base, size, {{0, size}}});
        held_ += size;
        return take(chunks_.back(), need, out);
    }

    // Give back a range obtained from alloc (same size argument).
    void release(uintptr_t p, size_t bytes) {
        const size_t size = round(bytes);
        for (Chunk &c : chunks_) {
            if (p < c.base || p >= c.base + c.size) continue;
            size_t off = p - c.base, len = size;
            auto next = c.free.lower_bound(off);
            if (next != c.free.begin()) {
                auto prev = std::prev(next);
                if (prev->first + prev->second == off) {
                    off = prev->first;
                    len += prev->second;
                    c.free.erase(prev);
                }
            }
            if (next != c.free.end() && off + len == next->first) {
                len += next->second;
                c.free.erase(next);
            }
            c.free[off] = len;
            in_use_ -= size;
            return;
        }
    }

    // Return every chunk (only valid when nothing is allocated).
    void reset() {
        for (Chunk &c : chunks_) shrink_(c.base);
        chunks_.clear();
        held_ = 0;
    }

    size_t in_use() const { return in_use_; }
    size_t held() const { return held_; }
    size_t budget() const { return budget_; }
    size_t chunks() const { return chunks_.size(); }

  private:
    struct Chunk {
        uintptr_t base;
        size_t size;
        std::map<size_t, size_t> free;   // offset -> length
    };

    bool take(Chunk &c, size_t need, uintptr_t *out) {
        for (auto it = c.free.begin(); it != c.free.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, len = it->second;
            c.free.erase(it);
            if (len > need) c.free[off + need] = len - need;
            *out = c.base + off;
            in_use_ += need;
            return true;
        }
        return false;
    }

    size_t budget_, chunk_;
    GrowFn grow_;
    ShrinkFn shrink_;
    std::vector<Chunk> chunks_;
    size_t held_ = 0, in_use_ = 0;
};

// Requests waiting for admission, earliest arrival first (ties in submission order).  A
// request is eligible once its arrival time has passed.
template <class T>
class ArrivalQueue {
  public:
    void push(double arrival, const T &v) { q_.push(Entry{arrival, seq_++, v}); }
    bool empty() const { return q_.empty(); }
    size_t size() const { return q_.size(); }
    // Earliest arrival, or +inf when empty.
    double next_arrival() const { return q_.empty() ? 1e300 : q_.top().arrival; }
    bool ready(double now) const { return !q_.empty() && q_.top().arrival <= now; }
    const T &front() const { return q_.top().v; }
    double front_arrival() const { return q_.top().arrival; }
    void pop() { q_.pop(); }

  private:
    struct Entry {
        double arrival;
        uint64_t seq;
        T v;
        bool operator<(const Entry &o) const {   // max-heap: invert for earliest first
            return arrival != o.arrival ? arrival > o.arrival : seq > o.seq;
        }
    };
    std::priority_queue<Entry> q_;
    uint64_t seq_ = 0;
};

// Admission of one batch: take eligible requests in arrival order while the batch has room
// (request count, tile items) and the arena can hold the request's packed operands.  The
// first request that does not fit ends the batch (no overtaking, so no request starves).
// `items_of(v)` gives a request's tile count, `bytes_of(v)` its arena bytes; admitted
// requests are appended to `out` with their arena address.  Returns false when the head
// request cannot be placed even though nothing is in flight (the caller then resets the
// arena and retries).
template <class T, class ItemsFn, class BytesFn>
bool admit_batch(ArrivalQueue<T> &queue, Arena &arena, double now, int max_requests, size_t max_items,
                 ItemsFn items_of, BytesFn bytes_of, std::vector<std::pair<T, uintptr_t>> *out, bool idle) {
    size_t items = 0;
    while (queue.ready(now) && (int)out->size() < max_requests) {
        const T &v = queue.front();
        const size_t it = items_of(v);
        if (!out->empty() && items + it > max_items) break;
        uintptr_t p = 0;
        if (!arena.alloc(bytes_of(v), &p)) return !(idle && out->empty());
        out->push_back(std::make_pair(v, p));
        items += it;
        queue.pop();
    }
    return true;
}

}  // namespace gfq
