// admission.h -- the roll-out server's memory and admission policy, host-only
// C++ (no HIP), so that it can be tested on the CPU: a first-fit
// sub-allocator over the caller's device arena (the HBM admission budget)
// and the order in which queued requests are admitted.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>

namespace wsx {

inline size_t arena_align(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit sub-allocator over [0, size) in 256-byte granules; freed
// neighbours merge. Offsets only: the caller adds its base pointer.
class Arena {
public:
    void init(size_t size) {
        size_ = size;
        free_.clear();
        in_use_ = peak_ = 0;
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = arena_align(bytes);
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, next = it->first + bytes;
            free_.erase(it);
            if (rest) free_[next] = rest;
            in_use_ += bytes;
            peak_ = std::max(peak_, in_use_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = arena_align(bytes);
        if (bytes == 0) bytes = 256;
        in_use_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }
    size_t in_use() const { return in_use_; }
    size_t peak() const { return peak_; }
    size_t free_blocks() const { return free_.size(); }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }

private:
    size_t size_ = 0;
    std::map<size_t, size_t> free_;
    size_t in_use_ = 0, peak_ = 0;
};

// One admission pass over the queue (ids in arrival order): try(id) admits a
// request, or rejects it for good, and returns true (it leaves the queue), or
// returns false when it does not fit yet (it stays queued). A request that
// has waited longer than `head_wait_ms` at the head of the queue stops later
// ones from overtaking it, so a large request is not starved by a stream of
// small ones. waited_ms(id) is the time since the request was submitted.
// Returns whether any request left the queue.
template <class Try, class Waited>
bool admit_in_order(std::deque<int64_t>& queue, double head_wait_ms, Try&& try_one,
                    Waited&& waited_ms) {
    bool any = false;
    for (auto it = queue.begin(); it != queue.end();) {
        const bool head = it == queue.begin();
        if (try_one(*it)) {
            it = queue.erase(it);
            any = true;
        } else {
            if (head && waited_ms(*it) > head_wait_ms) break;
            ++it;
        }
    }
    return any;
}

}  // namespace wsx
