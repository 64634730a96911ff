// Host-side bookkeeping with no HIP calls: the serving arena's allocator and
// the stream's window cutter. Kept free of the runtime so a host-only build
// (sanitizers, unit checks) can exercise them.
#pragma once

#include <algorithm>
#include <cstdint>
#include <iterator>
#include <map>
#include <vector>

namespace dnatok {

// First-fit allocator over a byte range [0, size), free blocks coalesced.
// Blocks are rounded up to `align` bytes (a power of two).
class Arena {
  public:
    explicit Arena(int64_t align = 256) : align_(align) {}
    void reset(int64_t size) {
        free_.clear();
        if (size > 0) free_[0] = size;
        used_ = peak_ = 0;
    }
    int64_t round(int64_t size) const { return (std::max<int64_t>(size, 1) + align_ - 1) / align_ * align_; }
    // Offset of a block of `size` bytes, or -1.
    int64_t alloc(int64_t size) {
        size = round(size);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < size) continue;
            const int64_t off = it->first, rest = it->second - size;
            free_.erase(it);
            if (rest > 0) free_[off + size] = rest;
            used_ += size;
            peak_ = std::max(peak_, used_);
            return off;
        }
        return -1;
    }
    // Return a block given out by alloc with the same size.
    void release(int64_t off, int64_t size) {
        size = round(size);
        used_ -= size;
        auto it = free_.emplace(off, size).first;
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
    int64_t used() const { return used_; }
    int64_t peak() const { return peak_; }
    // Free blocks (offset -> size), for checks.
    const std::map<int64_t, int64_t> &free_blocks() const { return free_; }

  private:
    int64_t align_;
    std::map<int64_t, int64_t> free_;
    int64_t used_ = 0, peak_ = 0;
};

// Windows of a stream chunk. The bytes S = carry ++ chunk are addressed from
// the carry's first byte: `carry` bytes of the unfinished window, then the
// chunk's `nbytes`. Records end at ends[0..n_ends) (chunk coordinates,
// non-decreasing within [0, nbytes]); windows are `window` bytes counted from
// each record start, a record's last window being shorter. Writes the window
// bounds that S completes (cuts[0] = 0, then one entry per window end) and
// returns the start of the unfinished window (the next carry begins there).
inline int64_t cut_windows(int64_t carry, int64_t nbytes, int64_t window, const int64_t *ends, int32_t n_ends,
                           std::vector<int64_t> &cuts) {
    const int64_t slen = carry + nbytes;
    cuts.clear();
    cuts.reserve((size_t)(slen / window + n_ends + 2));
    cuts.push_back(0);
    int64_t cur = 0;
    int32_t ei = 0;
    for (;;) {
        const int64_t target = cur + window;
        const int64_t re = (ei < n_ends) ? ends[ei] + carry : INT64_MAX;
        if (re <= target) {
            if (re > cur) {
                cuts.push_back(re);
                cur = re;
            }
            ++ei;
        } else if (target <= slen) {
            cuts.push_back(target);
            cur = target;
        } else {
            break;
        }
    }
    return cur;
}

}  // namespace dnatok
