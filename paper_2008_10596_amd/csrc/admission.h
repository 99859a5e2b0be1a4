// admission.h -- the serving loop's admission policy and staging arena, free
// of HIP calls so that the host logic can be exercised on its own (the CPU
// tests drive it under AddressSanitizer and UndefinedBehaviorSanitizer).
//
// A request is admitted when a slot is free and its device staging block fits
// the arena.  A checkpoint also needs pinned host memory for the image it
// produces: it is admitted only while the pinned bytes held by images
// (anywhere in the process), plus the charges of admitted checkpoints, plus
// its own charge stay within the host budget.  Requests are taken in arrival
// order, with one exception: a checkpoint that waits for host memory lets the
// restores behind it pass (they need no new host memory, and finishing them
// is what lets a caller release older images), while the checkpoints behind
// it keep waiting in order.  A request whose device block does not fit stops
// admission for everyone behind it.
#pragma once

#include <cstdint>
#include <map>

namespace ckpt {

// First-fit allocator over the offsets [0, size) of one device block.
class ArenaMap {
public:
    void reset(uint64_t size)
    {
        free_.clear();
        if (size)
            free_[0] = size;
        size_ = size;
        used_ = 0;
    }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    bool fits(uint64_t bytes) const
    {
        for (const auto &h : free_)
            if (h.second >= bytes)
                return true;
        return false;
    }
    // offset of a block of `bytes`, or UINT64_MAX when no hole is large enough
    uint64_t alloc(uint64_t bytes)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                const uint64_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest)
                    free_[off + bytes] = rest;
                used_ += bytes;
                return off;
            }
        return UINT64_MAX;
    }
    void free(uint64_t off, uint64_t bytes)
    {
        if (!bytes)
            return;
        used_ -= bytes;
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
    // The holes, for consistency checks: start -> bytes.
    const std::map<uint64_t, uint64_t> &holes() const { return free_; }

private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t size_ = 0, used_ = 0;
};

// What admission needs to know of a queued request.
struct AdmitInfo {
    bool checkpoint = false;   // produces an image in pinned host memory
    uint64_t dev_bytes = 0;    // device staging block
    uint64_t host_bytes = 0;   // checkpoint: the most pinned memory its image can take
};

struct AdmitState {
    uint32_t max_active = 16;
    uint32_t n_active = 0;
    uint64_t host_budget = 0;     // 0: no host limit
    uint64_t host_reserved = 0;   // charges of admitted, unfinished checkpoints
};

// Position in `queue` (arrival order) of the next request to admit, or -1.
// host_live: pinned bytes held now by images and buffers outside the
// reservations.  *host_blocked is set when a checkpoint waits for host memory
// (the caller then polls again after host memory may have been released).
template <class Queue, class InfoOf>
long next_admissible(const Queue &queue, const AdmitState &st, const ArenaMap &arena, uint64_t host_live,
                     InfoOf info_of, bool *host_blocked)
{
    *host_blocked = false;
    if (st.n_active >= st.max_active)
        return -1;
    long i = 0;
    for (auto it = queue.begin(); it != queue.end(); ++it, ++i) {
        const AdmitInfo r = info_of(*it);
        if (r.checkpoint) {
            if (*host_blocked)
                continue;   // checkpoints keep their order behind a waiting one
            if (st.host_budget && host_live + st.host_reserved + r.host_bytes > st.host_budget) {
                *host_blocked = true;
                continue;
            }
        }
        return arena.fits(r.dev_bytes) ? i : -1;
    }
    return -1;
}

}  // namespace ckpt
