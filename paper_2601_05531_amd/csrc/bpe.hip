// Ranked-merge BPE on the device: vocabulary tables and the encode pipeline.
//
// Paper: BPE / data-driven subwords (introduction, table of genomic
// tokenization schemes; the BPE of Sennrich et al. it cites); DNATok keeps
// "identical token IDs and segmentation" (Discussion, accuracy and
// algorithmic neutrality) and BPE is one of the vocabularies it accelerates.
//
// Semantics (as the oracle): case folded; each maximal ACGT run is
// segmented on its own (N -> 9 and other bytes -> UNK are barriers); within a
// run, repeatedly the lowest-ranked adjacent pair is replaced everywhere,
// left to right, by the merge's id 10 + rank.
//
// Device form: for a well-formed table (operands are bases or earlier
// merges; no pair twice) a merge's new symbol only forms pairs of higher
// rank, so the rank applied in each round strictly increases. A block keeps
// a histogram of the ranks of all current adjacent pairs and walks it
// forward: each round takes the next rank present, merges all its
// non-overlapping occurrences in parallel (runs of (X, X) pairs resolved by
// parity, leftmost first), updates the histogram for the pairs destroyed and
// created, and compacts the symbols. Barriers never merge, so a block can
// segment many runs at once.
//
// Pipeline (all on the caller's stream):
//  1. item plan: rows are cut into nominal items of S bytes; item offsets are
//     a row scan of ceil(L / S). Item j of a row starts just after the first
//     barrier at or after byte j * S (or at the row end), so no run is split.
//  2. k_bpe_merge: persistent 1024-thread blocks take items by ticket; the
//     pair -> rank hash and the rank histogram sit in LDS, the symbols too
//     unless a segment is longer than the LDS budget (then global scratch).
//  3. k_scan_counts: item token counts -> item positions (one-pass scan).
//  4. k_bpe_emit: CLS/SEP/pads/mask per row and body tokens per item into
//     the PACKED or PADDED output.
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "device.hpp"

namespace dnatok {

// ---- vocabulary tables ----------------------------------------------------------

int build_bpe_tables(dnatok_vocab *v) {
    BpeTables &t = v->bpe;
    const int32_t R = (int32_t)(v->h_merges.size() / 2);
    if (R > kBpeMaxMerges)
        return set_error(DNATOK_EVOCAB, "BPE tables hold at most %d merges (got %d)", kBpeMaxMerges, R);
    t.n_merges = R;
    const int32_t V = 10 + R;
    // expansions (uppercase bases) per id
    std::vector<int32_t> len(V, 1);
    std::vector<int64_t> off(V, 0);
    for (int id = 0; id < 5; ++id) len[id] = 0;
    int64_t total = 0;
    for (int32_t r = 0; r < R; ++r) {
        int64_t L = (int64_t)len[v->h_merges[2 * r]] + len[v->h_merges[2 * r + 1]];
        if (L > (1 << 20)) return set_error(DNATOK_EVOCAB, "merge %d expands to more than 2^20 bases", r);
        len[10 + r] = (int32_t)L;
    }
    int32_t mx = 1;
    for (int32_t id = 0; id < V; ++id) {
        off[id] = total;
        total += len[id];
        if (len[id] > mx) mx = len[id];
    }
    std::vector<uint8_t> chars((size_t)(total > 0 ? total : 1));
    const char *B = "ACGTN";
    for (int32_t id = 5; id <= 9; ++id) chars[off[id]] = (uint8_t)B[id - 5];
    for (int32_t r = 0; r < R; ++r) {
        int32_t a = v->h_merges[2 * r], b = v->h_merges[2 * r + 1], id = 10 + r;
        std::copy(chars.begin() + off[a], chars.begin() + off[a] + len[a], chars.begin() + off[id]);
        std::copy(chars.begin() + off[b], chars.begin() + off[b] + len[b], chars.begin() + off[id] + len[a]);
    }
    v->max_token_bytes = mx;

    uint32_t slots = 16;
    while (slots < 2u * (uint32_t)(R > 0 ? R : 1)) slots <<= 1;
    std::vector<uint32_t> keys(slots, 0);
    std::vector<uint16_t> ranks(slots, 0);
    for (int32_t r = 0; r < R; ++r) {
        uint32_t a = (uint32_t)v->h_merges[2 * r], b = (uint32_t)v->h_merges[2 * r + 1];
        uint32_t s = bpe_pair_hash(a, b) & (slots - 1);
        while (keys[s]) s = (s + 1) & (slots - 1);
        keys[s] = (a << 16) | b;
        ranks[s] = (uint16_t)r;
    }
    t.slots = slots;

    void *p = nullptr;
    DNATOK_HIP(hipMalloc(&p, sizeof(uint32_t) * slots));
    t.d_hkey = static_cast<uint32_t *>(p);
    DNATOK_HIP(hipMemcpy(t.d_hkey, keys.data(), sizeof(uint32_t) * slots, hipMemcpyHostToDevice));
    DNATOK_HIP(hipMalloc(&p, sizeof(uint16_t) * slots));
    t.d_hrank = static_cast<uint16_t *>(p);
    DNATOK_HIP(hipMemcpy(t.d_hrank, ranks.data(), sizeof(uint16_t) * slots, hipMemcpyHostToDevice));
    DNATOK_HIP(hipMalloc(&p, sizeof(int32_t) * 2 * (size_t)(R > 0 ? R : 1)));
    t.d_merges = static_cast<int32_t *>(p);
    if (R > 0)
        DNATOK_HIP(hipMemcpy(t.d_merges, v->h_merges.data(), sizeof(int32_t) * 2 * (size_t)R, hipMemcpyHostToDevice));
    DNATOK_HIP(hipMalloc(&p, sizeof(int32_t) * (size_t)V));
    t.d_tok_len = static_cast<int32_t *>(p);
    DNATOK_HIP(hipMemcpy(t.d_tok_len, len.data(), sizeof(int32_t) * (size_t)V, hipMemcpyHostToDevice));
    DNATOK_HIP(hipMalloc(&p, sizeof(int64_t) * (size_t)V));
    t.d_tok_off = static_cast<int64_t *>(p);
    DNATOK_HIP(hipMemcpy(t.d_tok_off, off.data(), sizeof(int64_t) * (size_t)V, hipMemcpyHostToDevice));
    DNATOK_HIP(hipMalloc(&p, chars.size()));
    t.d_tok_chars = static_cast<uint8_t *>(p);
    DNATOK_HIP(hipMemcpy(t.d_tok_chars, chars.data(), chars.size(), hipMemcpyHostToDevice));
    return DNATOK_OK;
}

void free_bpe_tables(dnatok_vocab *v) {
    BpeTables &t = v->bpe;
    if (t.d_hkey) (void)hipFree(t.d_hkey);
    if (t.d_hrank) (void)hipFree(t.d_hrank);
    if (t.d_merges) (void)hipFree(t.d_merges);
    if (t.d_tok_len) (void)hipFree(t.d_tok_len);
    if (t.d_tok_off) (void)hipFree(t.d_tok_off);
    if (t.d_tok_chars) (void)hipFree(t.d_tok_chars);
    t = BpeTables();
}

namespace {

constexpr int NTM = 1024;          // merge kernel block
constexpr int NTE = 256;           // scan / emit blocks
constexpr int32_t kItemBytes = 8192;  // nominal item length S
constexpr int kScanPerThread = 16;
constexpr int64_t kScanUnit = (int64_t)NTE * kScanPerThread;
constexpr size_t kLdsBudget = 156 * 1024;

__device__ __forceinline__ bool is_base_byte(uint8_t b) {
    const uint8_t f = b | 0x20;
    return f == 'a' || f == 'c' || f == 'g' || f == 't';
}

__device__ __forceinline__ uint16_t symbol_of(uint8_t b) {
    switch (b | 0x20) {
    case 'a': return 5;
    case 'c': return 6;
    case 'g': return 7;
    case 't': return 8;
    case 'n': return 9;
    default: return DNATOK_ID_UNK;
    }
}

struct MergeArgs {
    const uint8_t *bytes;
    int64_t nbytes;
    const int64_t *offs;
    int32_t n;
    const int64_t *item_off;  // [n + 1]
    int32_t S;
    uint16_t *symA;  // global scratch [nbytes]: final symbols of every item at its segment start
    uint16_t *symB;  // global scratch [nbytes]: second buffer for oversized segments
    int32_t *item_cnt;
    int64_t *item_start;
    int64_t max_items;
    const uint32_t *hkey;
    const uint16_t *hrank;
    uint32_t slots;
    const int32_t *merges;
    int32_t R;
    int32_t lmax;  // symbols per LDS buffer
    dev::TileQueue q;
};

// Item j >= 1 of row [off, end) may start only just after a barrier found
// in its own nominal window [off + j*S - 1, off + (j+1)*S - 1): the first
// such barrier q gives start q + 1; with none the item is empty (-1) and its
// bytes belong to the previous item. Starts therefore increase with j and
// consecutive non-empty items tile the row without splitting a run. All 64
// lanes of a wave call it.
__device__ int64_t item_start_probe(const uint8_t *bytes, int64_t off, int64_t end, int64_t j, int32_t S) {
    const int64_t x = off + j * (int64_t)S - 1;
    const int64_t lim = min(x + (int64_t)S, end);
    const int lane = threadIdx.x & (dev::kWave - 1);
    for (int64_t base = x; base < lim; base += dev::kWave * 16) {
        int64_t mine = INT64_MAX;
        const int64_t q0 = base + (int64_t)lane * 16;
        for (int u = 0; u < 16; ++u) {
            const int64_t q = q0 + u;
            if (q < lim && !is_base_byte(bytes[q])) {
                mine = q;
                break;
            }
        }
        const uint64_t hit = __ballot(mine != INT64_MAX);
        if (hit) return __shfl(mine, __builtin_ctzll(hit), dev::kWave) + 1;
    }
    return -1;
}

struct LdsTables {
    const uint32_t *hkey;
    const uint16_t *hrank;
    uint32_t mask;
};

__device__ __forceinline__ int32_t rank_of(const LdsTables &t, uint32_t x, uint32_t y) {
    if (x < 5 || x == 9 || y < 5 || y == 9) return -1;  // specials and barriers never merge
    const uint32_t key = (x << 16) | y;
    uint32_t s = bpe_pair_hash(x, y) & t.mask;
    for (;;) {
        const uint32_t k = t.hkey[s];
        if (k == key) return t.hrank[s];
        if (k == 0) return -1;
        s = (s + 1) & t.mask;
    }
}

// Chain state of a slice for the scan that finds, at each slice start, how
// many consecutive occurrences of an (X, X) pair end just before it.
struct Chain {
    int32_t full;  // every position of the slice starts an occurrence (empty: 1)
    int32_t tail;  // occurrences ending the slice
    int32_t len;   // slice length
};
__device__ __forceinline__ Chain chain_join(Chain a, Chain b) {
    return Chain{a.full & b.full, b.full ? a.tail + b.len : b.tail, a.len + b.len};
}

// Exclusive scan of Chain over the block's threads.
__device__ Chain chain_excl_scan(Chain c, Chain *s_wave) {
    const int lane = threadIdx.x & (dev::kWave - 1), w = threadIdx.x / dev::kWave;
    Chain inc = c;
#pragma unroll
    for (int d = 1; d < dev::kWave; d <<= 1) {
        Chain o;
        o.full = __shfl_up(inc.full, d, dev::kWave);
        o.tail = __shfl_up(inc.tail, d, dev::kWave);
        o.len = __shfl_up(inc.len, d, dev::kWave);
        if (lane >= d) inc = chain_join(o, inc);
    }
    if (lane == dev::kWave - 1) s_wave[w] = inc;
    __syncthreads();
    Chain pre{1, 0, 0};
    for (int i = 0; i < w; ++i) pre = chain_join(pre, s_wave[i]);
    // exclusive within the wave: inclusive of lane-1
    Chain lw;
    lw.full = __shfl_up(inc.full, 1, dev::kWave);
    lw.tail = __shfl_up(inc.tail, 1, dev::kWave);
    lw.len = __shfl_up(inc.len, 1, dev::kWave);
    __syncthreads();
    return lane == 0 ? pre : chain_join(pre, lw);
}

// Segment one item's symbols A[0, n) with B as the second buffer (both LDS
// or both global). Returns the final length; *in_a tells whether the result
// ended up in A.
template <class SymPtr>
__device__ int32_t merge_segment(SymPtr A, SymPtr B, int32_t n, const LdsTables &tab, int32_t *hist,
                                 const int32_t *merges, int32_t R, int64_t *s_tmp, Chain *s_chain, int32_t *s_rstar,
                                 bool *in_a) {
    const int tid = threadIdx.x;
    const int lane = tid & (dev::kWave - 1);
    bool a_is_a = true;
    for (int32_t r = tid; r < R; r += NTM) hist[r] = 0;
    __syncthreads();
    for (int32_t p = tid; p + 1 < n; p += NTM) {
        const int32_t r = rank_of(tab, A[p], A[p + 1]);
        if (r >= 0) atomicAdd(&hist[r], 1);
    }
    __syncthreads();
    int32_t cur = -1;
    for (;;) {
        if (tid < dev::kWave) {
            int32_t found = R;
            for (int32_t base = cur + 1; base < R; base += dev::kWave) {
                const int32_t idx = base + lane;
                const int32_t v = (idx < R) ? hist[idx] : 0;
                const uint64_t b = __ballot(v > 0);
                if (b) {
                    found = base + __builtin_ctzll(b);
                    break;
                }
            }
            if (lane == 0) *s_rstar = found;
        }
        __syncthreads();
        const int32_t rs = *s_rstar;
        if (rs >= R) break;
        cur = rs;
        const uint16_t L = (uint16_t)merges[2 * rs], Rr = (uint16_t)merges[2 * rs + 1];
        const uint16_t NEW = (uint16_t)(10 + rs);
        const bool chain = (L == Rr);
        const int32_t sl = (n + NTM - 1) / NTM;
        const int32_t a0 = min(n, tid * sl), a1 = min(n, a0 + sl);
        auto cand = [&](int32_t p) { return p >= 0 && p + 1 < n && A[p] == L && A[p + 1] == Rr; };

        int32_t carry = 0;  // occurrences ending at a0 - 1 (chains only)
        if (chain) {
            Chain c{1, 0, a1 - a0};
            for (int32_t p = a0; p < a1; ++p) {
                if (cand(p)) c.tail += 1;
                else {
                    c.tail = 0;
                    c.full = 0;
                }
            }
            carry = chain_excl_scan(c, s_chain).tail;
        }
        // merge start at p: an occurrence at an even offset from its chain's start
        const bool ms_before = (a0 >= 1) && cand(a0 - 1) && (!chain || ((carry - 1) & 1) == 0);

        // pass 1: pairs destroyed by this round, symbols kept
        int32_t kept = 0;
        {
            int32_t run = carry;
            bool prev = ms_before;
            for (int32_t p = a0; p < a1; ++p) {
                const bool c = cand(p);
                run = c ? run + 1 : 0;
                const bool ms = c && (!chain || ((run - 1) & 1) == 0);
                if (!prev) ++kept;
                if (ms) {
                    atomicSub(&hist[rs], 1);
                    if (p + 2 < n) {
                        const int32_t r2 = rank_of(tab, Rr, A[p + 2]);
                        if (r2 >= 0) atomicSub(&hist[r2], 1);
                    }
                    // the left pair belongs to this merge unless p-1 was consumed by a merge at p-2
                    const bool p2 = (p >= 2) && cand(p - 2) && (!chain || cand(p - 1));
                    if (p >= 1 && !p2) {
                        const int32_t r0 = rank_of(tab, A[p - 1], L);
                        if (r0 >= 0) atomicSub(&hist[r0], 1);
                    }
                }
                prev = ms;
            }
        }
        int64_t n2;
        const int32_t nb = (int32_t)dev::block_excl_scan<NTM>(kept, s_tmp, &n2);
        // pass 2: compact into B
        {
            int32_t run = carry, y = nb;
            bool prev = ms_before;
            for (int32_t p = a0; p < a1; ++p) {
                const bool c = cand(p);
                run = c ? run + 1 : 0;
                const bool ms = c && (!chain || ((run - 1) & 1) == 0);
                if (!prev) B[y++] = ms ? NEW : A[p];
                prev = ms;
            }
        }
        __syncthreads();
        // pass 3: pairs created around each new symbol (left end owns a pair)
        {
            int32_t run = carry, y = nb;
            bool prev = ms_before;
            for (int32_t p = a0; p < a1; ++p) {
                const bool c = cand(p);
                run = c ? run + 1 : 0;
                const bool ms = c && (!chain || ((run - 1) & 1) == 0);
                if (!prev) {
                    if (ms) {
                        if (y + 1 < n2) {
                            const int32_t r = rank_of(tab, NEW, B[y + 1]);
                            if (r >= 0) atomicAdd(&hist[r], 1);
                        }
                        if (y >= 1 && B[y - 1] != NEW) {
                            const int32_t r = rank_of(tab, B[y - 1], NEW);
                            if (r >= 0) atomicAdd(&hist[r], 1);
                        }
                    }
                    ++y;
                }
                prev = ms;
            }
        }
        __syncthreads();
        SymPtr t = A;
        A = B;
        B = t;
        a_is_a = !a_is_a;
        n = (int32_t)n2;
    }
    *in_a = a_is_a;
    return n;
}

__global__ __launch_bounds__(NTM) void k_bpe_merge(MergeArgs a) {
    extern __shared__ __align__(16) uint8_t dyn[];
    __shared__ int64_t s_tmp[NTM / dev::kWave + 1];
    __shared__ Chain s_chain[NTM / dev::kWave];
    __shared__ int32_t s_rstar;
    __shared__ int64_t s_ticket, s_c0, s_c1;

    uint32_t *hkey = reinterpret_cast<uint32_t *>(dyn);
    uint16_t *hrank = reinterpret_cast<uint16_t *>(hkey + a.slots);
    int32_t *hist = reinterpret_cast<int32_t *>(hrank + ((a.slots + 1) & ~1u));
    uint16_t *la = reinterpret_cast<uint16_t *>(hist + ((a.R + 1) & ~1));
    uint16_t *lb = la + a.lmax;
    const int tid = threadIdx.x;
    for (uint32_t s = tid; s < a.slots; s += NTM) {
        hkey[s] = a.hkey[s];
        hrank[s] = a.hrank[s];
    }
    const LdsTables tab{hkey, hrank, a.slots - 1};
    const int64_t total = min(a.item_off[a.n], a.max_items);
    __syncthreads();

    for (;;) {
        if (tid == 0) s_ticket = (int64_t)atomicAdd(a.q.hdr + 0, 1u);
        __syncthreads();
        const int64_t t = s_ticket;
        if (t >= total) break;
        if (tid < dev::kWave) {
            // row i: the last row whose first item is <= t
            const int64_t i1 = dev::wave_lower_bound(0, (int64_t)a.n + 1, [&](int64_t i) { return a.item_off[i] > t; });
            const int64_t i = i1 - 1, j = t - a.item_off[i], nj = a.item_off[i + 1] - a.item_off[i];
            int64_t off = a.offs[i], end = a.offs[i + 1];
            off = off < 0 ? 0 : (off > a.nbytes ? a.nbytes : off);
            end = end < off ? off : (end > a.nbytes ? a.nbytes : end);
            int64_t c0 = (j == 0) ? off : item_start_probe(a.bytes, off, end, j, a.S);
            int64_t c1 = c0;
            if (c0 >= 0) {
                c1 = end;
                for (int64_t jj = j + 1; jj < nj; ++jj) {
                    const int64_t b = item_start_probe(a.bytes, off, end, jj, a.S);
                    if (b >= 0) {
                        c1 = b;
                        break;
                    }
                }
            } else {
                c0 = c1 = 0;
            }
            if (tid == 0) {
                s_c0 = c0;
                s_c1 = c1 > c0 ? c1 : c0;
            }
        }
        __syncthreads();
        const int64_t c0 = s_c0, len = s_c1 - s_c0;
        int32_t nf = 0;
        if (len > 0) {
            if (len <= a.lmax) {
                for (int64_t p = tid; p < len; p += NTM) la[p] = symbol_of(a.bytes[c0 + p]);
                __syncthreads();
                bool in_a = true;
                nf = merge_segment(la, lb, (int32_t)len, tab, hist, a.merges, a.R, s_tmp, s_chain, &s_rstar, &in_a);
                const uint16_t *res = in_a ? la : lb;
                for (int32_t p = tid; p < nf; p += NTM) a.symA[c0 + p] = res[p];
            } else {
                uint16_t *ga = a.symA + c0, *gb = a.symB + c0;
                for (int64_t p = tid; p < len; p += NTM) ga[p] = symbol_of(a.bytes[c0 + p]);
                __syncthreads();
                bool in_a = true;
                nf = merge_segment(ga, gb, (int32_t)len, tab, hist, a.merges, a.R, s_tmp, s_chain, &s_rstar, &in_a);
                if (!in_a)
                    for (int32_t p = tid; p < nf; p += NTM) ga[p] = gb[p];
            }
        }
        if (tid == 0) {
            a.item_cnt[t] = nf;
            a.item_start[t] = c0;
        }
        __syncthreads();
    }
    if (tid == 0) dev::finish_block(a.q.hdr, false);
}

// ---- item count scan -------------------------------------------------------------------

struct ScanArgs {
    const int32_t *cnt;
    const int64_t *total_at;  // the number of items lives here (item_off[n])
    int64_t *pos;             // exclusive positions, pos[total] = sum
    int64_t max_items;
    int64_t nunits;
    dev::TileQueue q;
};

__global__ __launch_bounds__(NTE) void k_scan_counts(ScanArgs a) {
    __shared__ int64_t s_tmp[NTE / dev::kWave + 1];
    __shared__ int64_t s_unit, s_excl;
    const int tid = threadIdx.x;
    const uint32_t parity = dev::ld_relaxed32(a.q.hdr + 2);
    uint64_t *st = parity ? a.q.status1 : a.q.status0;
    uint64_t *st_other = parity ? a.q.status0 : a.q.status1;
    const int64_t total = min(*a.total_at, a.max_items);
    const int64_t units = (total + kScanUnit - 1) / kScanUnit > 0 ? (total + kScanUnit - 1) / kScanUnit : 1;
    for (;;) {
        if (tid == 0) s_unit = (int64_t)atomicAdd(a.q.hdr + 0, 1u);
        __syncthreads();
        const int64_t u = s_unit;
        __syncthreads();
        if (u >= a.nunits) break;
        for (int64_t j = u + (int64_t)tid * a.nunits; j < a.q.clear_n; j += (int64_t)NTE * a.nunits) st_other[j] = 0;
        if (u >= units) continue;  // beyond the items present: nothing to chain
        const int64_t i0 = u * kScanUnit + (int64_t)tid * kScanPerThread;
        int64_t v[kScanPerThread];
        int64_t mine = 0;
#pragma unroll
        for (int j = 0; j < kScanPerThread; ++j) {
            v[j] = (i0 + j < total) ? a.cnt[i0 + j] : 0;
            mine += v[j];
        }
        int64_t utot;
        const int64_t pre = dev::block_excl_scan<NTE>(mine, s_tmp, &utot);
        if (tid < dev::kWave) {
            if (tid == 0) dev::publish_aggregate(st, u, utot);
            const int64_t ex = dev::wave_lookback(st, u, utot);
            if (tid == 0) s_excl = ex;
        }
        __syncthreads();
        int64_t run = s_excl + pre;
#pragma unroll
        for (int j = 0; j < kScanPerThread; ++j) {
            if (i0 + j < total) a.pos[i0 + j] = run;
            run += v[j];
        }
        if (u == units - 1 && tid == 0) a.pos[total] = s_excl + utot;
        __syncthreads();
    }
    if (tid == 0) dev::finish_block(a.q.hdr);
}

// ---- emit ------------------------------------------------------------------------------

struct EmitArgs {
    const int64_t *offs;
    int32_t n;
    const int64_t *item_off;
    const int64_t *item_pos;
    const int32_t *item_cnt;
    const int64_t *item_start;
    int64_t max_items;
    const uint16_t *tok;  // symA
    int32_t *ids;
    int64_t cap;
    int64_t *out_offs;
    int8_t *mask;
    int32_t cls, padded, left;
    int32_t pad_id, cls_id, sep_id;
    int64_t W;
    int64_t base;
    uint32_t *err_hdr;
};

__global__ __launch_bounds__(NTE) void k_bpe_emit(EmitArgs a) {
    __shared__ uint32_t s_err;
    const int tid = threadIdx.x;
    if (tid == 0) s_err = 0;
    __syncthreads();
    uint32_t err = 0;
    // item indices are clamped to the scratch size (only malformed offsets reach it)
    auto first_item = [&](int64_t i) { return min(a.item_off[i], a.max_items); };
    const int64_t total = first_item(a.n);
    auto row_len = [&](int64_t i) { return a.item_pos[first_item(i + 1)] - a.item_pos[first_item(i)] + 2 * a.cls; };
    if (blockIdx.x == 0 && tid == 0 && a.n == 0) a.out_offs[0] = a.base;
    // rows: offsets, specials, pads
    for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
        const int64_t first = a.item_pos[first_item(i)];
        const int64_t len = row_len(i);
        if (tid == 0) {
            a.out_offs[i] = a.base + first + 2 * a.cls * i;
            if (i == a.n - 1) a.out_offs[a.n] = a.base + a.item_pos[total] + 2 * a.cls * a.n;
        }
        if (!a.padded) {
            if (a.cls && tid == 0) {
                const int64_t d = first + 2 * a.cls * i;
                if (d >= 0 && d < a.cap) a.ids[d] = a.cls_id;
                else err |= DNATOK_DERR_CAPACITY;
                if (d + len - 1 < a.cap) a.ids[d + len - 1] = a.sep_id;
                else err |= DNATOK_DERR_CAPACITY;
            }
            continue;
        }
        if (len > a.W) {
            err |= DNATOK_DERR_ROW_WIDTH;
            continue;
        }
        const int64_t lead = a.left ? a.W - len : 0;
        int32_t *row = a.ids + i * a.W;
        int8_t *mrow = a.mask + i * a.W;
        for (int64_t c = tid; c < a.W; c += NTE) {
            const int64_t tt = c - lead;
            if (tt < 0 || tt >= len) {
                row[c] = a.pad_id;
                mrow[c] = 0;
            } else if (a.cls && tt == 0) {
                row[c] = a.cls_id;
                mrow[c] = 1;
            } else if (a.cls && tt == len - 1) {
                row[c] = a.sep_id;
                mrow[c] = 1;
            }
        }
    }
    // items: body tokens
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int32_t cnt = a.item_cnt[t];
        if (cnt == 0) continue;
        // row of item t
        int64_t lo = 0, hi = a.n - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (a.item_off[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const int64_t i = lo;
        const uint16_t *src = a.tok + a.item_start[t];
        if (!a.padded) {
            const int64_t d = a.item_pos[t] + 2 * a.cls * i + a.cls;
            for (int32_t p = tid; p < cnt; p += NTE) {
                if (d + p < a.cap) a.ids[d + p] = src[p];
                else err |= DNATOK_DERR_CAPACITY;
            }
        } else {
            const int64_t len = row_len(i);
            if (len > a.W) continue;
            const int64_t lead = a.left ? a.W - len : 0;
            const int64_t d = i * a.W + lead + a.cls + (a.item_pos[t] - a.item_pos[first_item(i)]);
            for (int32_t p = tid; p < cnt; p += NTE) {
                a.ids[d + p] = src[p];
                a.mask[d + p] = 1;
            }
        }
    }
    if (err) atomicOr(&s_err, err);
    __syncthreads();
    if (tid == 0 && s_err) dev::raise_error(a.err_hdr, s_err);
}

}  // namespace

int launch_bpe_encode(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                      int32_t n, int32_t *d_ids, int64_t cap, int64_t *d_out_offsets, int8_t *d_mask,
                      const dnatok_encode_opts &o, hipStream_t stream) {
    const BpeTables &bt = v->bpe;
    const int32_t R = bt.n_merges;
    if (R > kBpeMaxMerges) return set_error(DNATOK_EVOCAB, "device BPE supports up to %d merges", kBpeMaxMerges);
    const int64_t max_items = nbytes / kItemBytes + (int64_t)n + 1;
    // scratch: symA, symB (uint16 per byte), item_off, item_cnt, item_start, item_pos
    auto al = [](int64_t x) { return (x + 255) / 256 * 256; };
    const int64_t sz_sym = al(2 * (nbytes + 1));
    const int64_t sz_ioff = al(8 * ((int64_t)n + 1));
    const int64_t sz_cnt = al(4 * max_items);
    const int64_t sz_start = al(8 * max_items);
    const int64_t sz_pos = al(8 * (max_items + 1));
    Workspace *ws = nullptr;
    const int64_t units_rows = std::max<int64_t>(1, ((int64_t)n + 4095) / 4096);
    const int64_t units_items = std::max<int64_t>(1, (max_items + kScanUnit - 1) / kScanUnit);
    int rc = get_workspace(stream, std::max(units_rows, units_items), &ws);
    if (rc) return rc;
    rc = ensure_scratch(ws, 2 * sz_sym + sz_ioff + sz_cnt + sz_start + sz_pos);
    if (rc) return rc;
    uint8_t *sp = ws->d_scratch;
    uint16_t *symA = reinterpret_cast<uint16_t *>(sp);
    uint16_t *symB = reinterpret_cast<uint16_t *>(sp + sz_sym);
    int64_t *item_off = reinterpret_cast<int64_t *>(sp + 2 * sz_sym);
    int32_t *item_cnt = reinterpret_cast<int32_t *>(sp + 2 * sz_sym + sz_ioff);
    int64_t *item_start = reinterpret_cast<int64_t *>(sp + 2 * sz_sym + sz_ioff + sz_cnt);
    int64_t *item_pos = reinterpret_cast<int64_t *>(sp + 2 * sz_sym + sz_ioff + sz_cnt + sz_start);

    // 1. item plan
    rc = launch_rowscan(d_offsets, n, nbytes, item_off, kItemBytes, 0, stream);
    if (rc) return rc;

    // 2. merges
    MergeArgs m;
    m.bytes = d_bytes;
    m.nbytes = nbytes;
    m.offs = d_offsets;
    m.n = n;
    m.item_off = item_off;
    m.S = kItemBytes;
    m.symA = symA;
    m.symB = symB;
    m.item_cnt = item_cnt;
    m.item_start = item_start;
    m.max_items = max_items;
    m.hkey = bt.d_hkey;
    m.hrank = bt.d_hrank;
    m.slots = bt.slots;
    m.merges = bt.d_merges;
    m.R = R;
    const size_t tables = (size_t)bt.slots * 4 + (size_t)((bt.slots + 1) & ~1u) * 2 + (size_t)((R + 1) & ~1) * 4;
    int64_t lmax = (int64_t)((kLdsBudget - tables) / 4);
    lmax = lmax / NTM * NTM;
    if (lmax < NTM) return set_error(DNATOK_EVOCAB, "BPE tables leave no room for symbols in LDS");
    m.lmax = (int32_t)lmax;
    const size_t dyn = tables + 4 * (size_t)lmax;
    m.q.hdr = ws->d_hdr;
    m.q.status0 = ws->d_status;
    m.q.status1 = ws->d_status + ws->cap;
    m.q.clear_n = ws->high_water;
    DNATOK_HIP(hipFuncSetAttribute((const void *)k_bpe_merge, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    int64_t grid = std::min<int64_t>(max_items, (int64_t)device_cu_count());
    hipLaunchKernelGGL(k_bpe_merge, dim3((unsigned)grid), dim3(NTM), dyn, stream, m);
    DNATOK_HIP(hipGetLastError());

    // 3. item positions
    ScanArgs sa;
    sa.cnt = item_cnt;
    sa.total_at = item_off + n;
    sa.pos = item_pos;
    sa.max_items = max_items;
    sa.nunits = units_items;
    sa.q.hdr = ws->d_hdr;
    sa.q.status0 = ws->d_status;
    sa.q.status1 = ws->d_status + ws->cap;
    if (units_items > ws->high_water) ws->high_water = units_items;
    sa.q.clear_n = ws->high_water;
    int per_cu = 0;
    DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_scan_counts, NTE, 0));
    int64_t g2 = std::min<int64_t>(units_items, (int64_t)device_cu_count() * std::max(per_cu, 1));
    hipLaunchKernelGGL(k_scan_counts, dim3((unsigned)g2), dim3(NTE), 0, stream, sa);
    DNATOK_HIP(hipGetLastError());

    // 4. emit
    EmitArgs e;
    e.offs = d_offsets;
    e.n = n;
    e.item_off = item_off;
    e.item_pos = item_pos;
    e.item_cnt = item_cnt;
    e.item_start = item_start;
    e.max_items = max_items;
    e.tok = symA;
    e.ids = d_ids;
    e.cap = cap;
    e.out_offs = d_out_offsets;
    e.mask = d_mask;
    e.cls = o.add_cls_sep ? 1 : 0;
    e.padded = (o.layout == DNATOK_PADDED) ? 1 : 0;
    e.left = (o.pad_side == DNATOK_PAD_LEFT) ? 1 : 0;
    e.pad_id = v->pad_id;
    e.cls_id = v->cls_id;
    e.sep_id = v->sep_id;
    e.W = e.padded ? o.pad_to : 0;
    e.base = o.offset_base;
    e.err_hdr = ws->d_hdr;
    int64_t g3 = std::max<int64_t>(1, std::min<int64_t>(std::max<int64_t>(n, max_items), (int64_t)device_cu_count() * 8));
    hipLaunchKernelGGL(k_bpe_emit, dim3((unsigned)g3), dim3(NTE), 0, stream, e);
    DNATOK_HIP(hipGetLastError());
    return DNATOK_OK;
}

}  // namespace dnatok
