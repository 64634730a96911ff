// Host-only driver for the sanitizer test: the serving arena's allocator and
// the stream's window cutter (paper_2601_05531_amd/csrc/hostbook.hpp) under
// random operation sequences, each checked against a brute-force model.
// Built with AddressSanitizer / UndefinedBehaviorSanitizer; prints "ok".
#include <cstdio>
#include <random>
#include <vector>

#include "hostbook.hpp"

static int failures = 0;
#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                     \
        }                                                                   \
    } while (0)

// Arena: live blocks never overlap and lie inside the range, used() is
// their rounded sum, and once everything is released the range is one free
// block again.
static void arena_random(uint64_t seed, int64_t size) {
    std::mt19937_64 rng(seed);
    dnatok::Arena a(256);
    a.reset(size);
    struct Blk { int64_t off, size; };
    std::vector<Blk> live;
    for (int step = 0; step < 20000; ++step) {
        if (live.empty() || rng() % 3 != 0) {
            const int64_t want = (int64_t)(rng() % 5000);
            const int64_t off = a.alloc(want);
            if (off < 0) continue;
            const int64_t r = a.round(want);
            CHECK(off % 256 == 0 && off >= 0 && off + r <= size);
            for (const Blk &b : live) CHECK(off + r <= b.off || b.off + a.round(b.size) <= off);
            live.push_back({off, want});
        } else {
            const size_t i = (size_t)(rng() % live.size());
            a.release(live[i].off, live[i].size);
            live[i] = live.back();
            live.pop_back();
        }
        int64_t used = 0;
        for (const Blk &b : live) used += a.round(b.size);
        CHECK(used == a.used());
    }
    for (const Blk &b : live) a.release(b.off, b.size);
    CHECK(a.used() == 0);
    CHECK(a.free_blocks().size() == 1 && a.free_blocks().begin()->first == 0 &&
          a.free_blocks().begin()->second == size);
}

// Window cutter: pushing a byte stream in random chunks gives the same
// window bounds as cutting each record into windows from its start.
static void windows_random(uint64_t seed) {
    std::mt19937_64 rng(seed);
    const int64_t window = 1 + (int64_t)(rng() % 50);
    std::vector<int64_t> recs;
    int64_t total = 0;
    const int nrec = 1 + (int)(rng() % 12);
    for (int r = 0; r < nrec; ++r) {
        const int64_t L = (rng() % 4 == 0) ? 0 : (int64_t)(rng() % 300);
        recs.push_back(L);
        total += L;
    }
    // expected: absolute window ends
    std::vector<int64_t> want;
    int64_t pos = 0;
    for (int64_t L : recs) {
        for (int64_t s = 0; s < L; s += window) want.push_back(pos + std::min(s + window, L));
        pos += L;
    }
    // record ends (absolute)
    std::vector<int64_t> ends;
    pos = 0;
    for (int64_t L : recs) {
        pos += L;
        ends.push_back(pos);
    }
    // push in random chunks; a record ending exactly at a chunk start is
    // reported by the earlier chunk
    std::vector<int64_t> got;
    int64_t carry_start = 0, c0 = 0;
    std::vector<int64_t> cuts;
    size_t ei = 0;
    while (c0 < total || (c0 == 0 && total == 0)) {
        const int64_t chunk = 1 + (int64_t)(rng() % 97);
        const int64_t c1 = std::min(total, c0 + chunk);
        std::vector<int64_t> ce;
        while (ei < ends.size() && ends[ei] <= c1) {
            if (ends[ei] > c0 || (ends[ei] == c0 && c0 == 0)) ce.push_back(ends[ei] - c0);
            ++ei;
        }
        const int64_t carry = c0 - carry_start;
        const int64_t cur = dnatok::cut_windows(carry, c1 - c0, window, ce.data(), (int32_t)ce.size(), cuts);
        CHECK(cuts.front() == 0);
        for (size_t j = 1; j < cuts.size(); ++j) {
            CHECK(cuts[j] > cuts[j - 1] && cuts[j] - cuts[j - 1] <= window);
            got.push_back(carry_start + cuts[j]);
        }
        CHECK(cur == cuts.back() && cur <= carry + (c1 - c0));
        carry_start += cur;
        if (total == 0) break;
        c0 = c1;
    }
    // flush: the unfinished window becomes the last one
    if (carry_start < total) got.push_back(total);
    CHECK(got == want);
}

int main() {
    for (uint64_t s = 1; s <= 6; ++s) arena_random(s, (int64_t)(s * 300000));
    for (uint64_t s = 1; s <= 3000; ++s) windows_random(s);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
