// Host-side bookkeeping with no HIP calls: the serving arena's allocator and
// the stream's window cutter. Kept free of the runtime so a host-only build
// (sanitizers, unit checks) can exercise them.
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <iterator>
#include <map>
#include <mutex>
#include <thread>
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

// A fixed set of worker threads that runs one parallel loop at a time: run()
// hands out parts [0, parts) to the workers and the calling thread and
// returns when every part is done. Created once per owner and reused, so a
// call costs a wake-up, not a thread start.
class WorkerPool {
  public:
    explicit WorkerPool(int threads) {
        const int extra = std::max(threads, 1) - 1;
        for (int i = 0; i < extra; ++i) workers_.emplace_back([this] { loop(); });
    }
    ~WorkerPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : workers_) t.join();
    }
    WorkerPool(const WorkerPool &) = delete;
    WorkerPool &operator=(const WorkerPool &) = delete;
    int size() const { return (int)workers_.size() + 1; }

    void run(int parts, const std::function<void(int)> &fn) {
        if (parts <= 0) return;
        if (workers_.empty() || parts == 1) {
            for (int p = 0; p < parts; ++p) fn(p);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            fn_ = &fn;
            parts_ = parts;
            next_.store(0);
            left_ = parts;
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [this] { return left_ == 0; });
        fn_ = nullptr;
    }

  private:
    void work() {
        for (;;) {
            const int p = next_.fetch_add(1);
            if (p >= parts_) return;
            (*fn_)(p);
            std::lock_guard<std::mutex> lk(mu_);
            if (--left_ == 0) done_cv_.notify_all();
        }
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
            }
            work();
        }
    }
    std::vector<std::thread> workers_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int)> *fn_ = nullptr;
    int parts_ = 0;
    std::atomic<int> next_{0};
    int left_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

// The host-side IDs path of the EmbedFromStrings algorithm for rows
// [r0, r1) of equal-length strings: each byte of a row of row_len bytes is
// mapped through the 256-entry table, and a row is left-padded with pad_id
// to token_len ids (>= row_len), the original positions right-aligned. Row i
// goes to dst[i * token_len ..).
template <class T>
inline void map_rows_to_ids(const int32_t *lut, int32_t pad_id, const uint8_t *src, int64_t r0, int64_t r1,
                            int64_t row_len, int64_t token_len, T *dst) {
    T table[256];
    for (int b = 0; b < 256; ++b) table[b] = (T)lut[b];
    const int64_t lead = token_len - row_len;
    for (int64_t i = r0; i < r1; ++i) {
        const uint8_t *s = src + i * row_len;
        T *d = dst + i * token_len;
        for (int64_t j = 0; j < lead; ++j) d[j] = (T)pad_id;
        d += lead;
        for (int64_t j = 0; j < row_len; ++j) d[j] = table[s[j]];
    }
}

}  // namespace dnatok
