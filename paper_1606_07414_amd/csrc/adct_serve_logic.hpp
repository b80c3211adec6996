// Host-side policy of the server, free of HIP: the device-memory pool,
// first-come-first-served admission, and latency percentiles.  The server
// and the simulation entry points used by the tests share this code.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

namespace adct {

// First-fit allocator over [0, capacity) in 256-byte granules; freed blocks
// coalesce with their neighbours.
class Pool {
  public:
    static int64_t round_up(int64_t bytes) { return (bytes + 255) & ~(int64_t)255; }

    explicit Pool(int64_t capacity) : cap_(capacity & ~(int64_t)255) {
        if (cap_ > 0) free_[0] = cap_;
    }

    // Offset of a block of at least `bytes`, or -1 when no free block is large enough.
    int64_t alloc(int64_t bytes) {
        const int64_t need = round_up(bytes < 1 ? 1 : bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                const int64_t off = it->first, rest = it->second - need;
                free_.erase(it);
                if (rest) free_[off + need] = rest;
                used_ += need;
                high_ = std::max(high_, used_);
                return off;
            }
        }
        return -1;
    }

    void release(int64_t off, int64_t bytes) {
        int64_t size = round_up(bytes < 1 ? 1 : bytes);
        used_ -= size;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + size == next->first) {
            size += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += size;
                return;
            }
        }
        free_[off] = size;
    }

    int64_t capacity() const { return cap_; }
    int64_t used() const { return used_; }
    int64_t high_water() const { return high_; }
    bool fits_ever(int64_t bytes) const { return round_up(bytes) <= cap_; }

  private:
    int64_t cap_;
    int64_t used_ = 0, high_ = 0;
    std::map<int64_t, int64_t> free_;
};

// One admission pass: requests are considered strictly in submission order
// (the head blocks the ones behind it); a request is admitted once it has
// arrived, fewer than max_inflight are held, and the pool can place it.
// `arrival(i)`, `bytes(i)` describe request i; `on_admit(i, offset)` takes
// it.  Returns the new head index.
template <typename ArrivalFn, typename BytesFn, typename SkipFn, typename AdmitFn>
int64_t admit_in_order(int64_t head, int64_t n, int64_t now, int64_t& inflight, int64_t max_inflight, Pool& pool,
                       ArrivalFn arrival, BytesFn bytes, SkipFn skip, AdmitFn on_admit) {
    while (head < n) {
        if (skip(head)) {
            ++head;
            continue;
        }
        if (arrival(head) > now || inflight >= max_inflight) break;
        const int64_t off = pool.alloc(bytes(head));
        if (off < 0) break;
        ++inflight;
        on_admit(head, off);
        ++head;
    }
    return head;
}

// Nearest-rank percentile (p in [0, 100]) of an unsorted sample.
inline double percentile(std::vector<double> v, double p) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double rank = std::ceil(p / 100.0 * (double)v.size());
    int64_t idx = (int64_t)rank - 1;
    if (idx < 0) idx = 0;
    if (idx >= (int64_t)v.size()) idx = (int64_t)v.size() - 1;
    return v[(size_t)idx];
}

}  // namespace adct
