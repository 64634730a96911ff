// Ranked-merge BPE on the device: vocabulary tables and the encode pipeline.
//
// Paper: BPE is one of the vocabularies of its table of genomic
// tokenization schemes (introduction, citing the subword BPE of Sennrich et
// al.), and the accelerated tokenizer must give the same ids and the same
// segmentation as the reference tokenizer (Discussion, accuracy and
// algorithmic neutrality).
//
// Semantics (as the oracle): case folded; each maximal ACGT run is segmented
// on its own (N -> 9 and other bytes -> UNK are barriers); within a run the
// lowest-ranked adjacent pair is replaced everywhere, left to right, by the
// merge's id 10 + rank, until no adjacent pair is in the table.
//
// Device form: for a well-formed table (operands are bases or earlier
// merges, no pair twice) a new symbol only forms pairs of higher rank, so
// the rank applied in each round strictly increases and every round merges
// all occurrences of one rank (runs of (X, X) pairs leftmost first).
//
// Pipeline (all on the caller's stream):
//  1. k_rowscan (encode.hip): rows are cut into nominal items of S bytes;
//     item offsets are the scan of ceil(L / S).
//  2. k_bpe_items: item j >= 1 of a row starts just after the first barrier
//     in its own nominal window (or is empty), so no ACGT run is split.
//  3. k_bpe_wave, once per length class: one wavefront per item, symbols,
//     pair ranks, an alive bitmap and a two-level min tree over the pair
//     ranks in LDS; a round touches only the blocks holding the current
//     rank. Classes trade waves per workgroup against symbols per wave.
//  4. k_bpe_block: items longer than the largest class, one 1024-thread
//     workgroup each, symbols in global scratch, a rank histogram in LDS.
//  5. k_scan_counts + k_bpe_emit: token counts -> positions -> ids.
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
    // expansions (uppercase bases) per id, for decode
    std::vector<int32_t> len(V, 1);
    std::vector<int64_t> off(V, 0);
    for (int id = 0; id < 5; ++id) len[id] = 0;
    for (int32_t r = 0; r < R; ++r) {
        int64_t L = (int64_t)len[v->h_merges[2 * r]] + len[v->h_merges[2 * r + 1]];
        if (L > (1 << 20)) return set_error(DNATOK_EVOCAB, "merge %d expands to more than 2^20 bases", r);
        len[10 + r] = (int32_t)L;
    }
    int64_t total = 0;
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

    // cuckoo table at load <= 0.8; grown by 5% and rebuilt if an insertion
    // walk does not settle
    std::vector<uint32_t> pair((size_t)(R > 0 ? R : 1), 0);
    for (int32_t r = 0; r < R; ++r)
        pair[r] = (uint32_t)v->h_merges[2 * r] | ((uint32_t)v->h_merges[2 * r + 1] << 16);
    uint32_t nbk = std::max<uint32_t>(1, (uint32_t)((R * 5 + 7) / 8));
    std::vector<uint32_t> bucket;
    for (int attempt = 0;; ++attempt) {
        if (attempt == 40) return set_error(DNATOK_EVOCAB, "could not build the pair table");
        bucket.assign((size_t)nbk * 4, 0);
        uint64_t rng = 0x2545F4914F6CDD1Dull + (uint64_t)attempt;
        bool ok = true;
        for (int32_t r = 0; r < R && ok; ++r) {
            uint32_t key = pair[r], rank = (uint32_t)r;
            uint32_t b1, b2;
            bpe_buckets(key, nbk, &b1, &b2);
            uint32_t cur = b1;
            bool placed = false;
            for (int kick = 0; kick < 500 && !placed; ++kick) {
                for (uint32_t c : {cur, cur == b1 ? b2 : b1}) {
                    for (int e = 0; e < 2 && !placed; ++e) {
                        if (bucket[(size_t)c * 4 + 2 * e] == 0) {
                            bucket[(size_t)c * 4 + 2 * e] = key;
                            bucket[(size_t)c * 4 + 2 * e + 1] = rank;
                            placed = true;
                        }
                    }
                    if (placed) break;
                }
                if (placed) break;
                // evict a random entry of the current bucket; move on to its other bucket
                rng ^= rng << 13;
                rng ^= rng >> 7;
                rng ^= rng << 17;
                const int e = (int)(rng & 1);
                std::swap(key, bucket[(size_t)cur * 4 + 2 * e]);
                std::swap(rank, bucket[(size_t)cur * 4 + 2 * e + 1]);
                bpe_buckets(key, nbk, &b1, &b2);
                cur = (cur == b1) ? b2 : b1;
            }
            ok = placed;
        }
        if (ok) break;
        nbk = nbk + nbk / 20 + 1;
    }
    t.nbk = nbk;

    void *p = nullptr;
    DNATOK_HIP(dev_alloc(&p, sizeof(uint32_t) * bucket.size()));
    t.d_bucket = static_cast<uint32_t *>(p);
    DNATOK_HIP(hipMemcpy(t.d_bucket, bucket.data(), sizeof(uint32_t) * bucket.size(), hipMemcpyHostToDevice));
    DNATOK_HIP(dev_alloc(&p, sizeof(uint32_t) * pair.size()));
    t.d_pair = static_cast<uint32_t *>(p);
    DNATOK_HIP(hipMemcpy(t.d_pair, pair.data(), sizeof(uint32_t) * pair.size(), hipMemcpyHostToDevice));
    DNATOK_HIP(dev_alloc(&p, sizeof(int32_t) * (size_t)V));
    t.d_tok_len = static_cast<int32_t *>(p);
    DNATOK_HIP(hipMemcpy(t.d_tok_len, len.data(), sizeof(int32_t) * (size_t)V, hipMemcpyHostToDevice));
    DNATOK_HIP(dev_alloc(&p, sizeof(int64_t) * (size_t)V));
    t.d_tok_off = static_cast<int64_t *>(p);
    DNATOK_HIP(hipMemcpy(t.d_tok_off, off.data(), sizeof(int64_t) * (size_t)V, hipMemcpyHostToDevice));
    DNATOK_HIP(dev_alloc(&p, chars.size()));
    t.d_tok_chars = static_cast<uint8_t *>(p);
    DNATOK_HIP(hipMemcpy(t.d_tok_chars, chars.data(), chars.size(), hipMemcpyHostToDevice));
    return DNATOK_OK;
}

void free_bpe_tables(dnatok_vocab *v) {
    BpeTables &t = v->bpe;
    if (t.d_bucket) (void)hipFree(t.d_bucket);
    if (t.d_pair) (void)hipFree(t.d_pair);
    if (t.d_tok_len) (void)hipFree(t.d_tok_len);
    if (t.d_tok_off) (void)hipFree(t.d_tok_off);
    if (t.d_tok_chars) (void)hipFree(t.d_tok_chars);
    t = BpeTables();
}

namespace {

constexpr int NTM = 1024;             // k_bpe_block workgroup
constexpr int NTE = 256;              // items / scan / emit workgroups
constexpr int kMaxWaves = 8;          // waves per k_bpe_wave workgroup
constexpr int kScanPerThread = 16;
constexpr int64_t kScanUnit = (int64_t)NTE * kScanPerThread;
constexpr size_t kLdsBytes = 160 * 1024;
constexpr size_t kLdsReserve = 2048;  // static LDS of the kernels
constexpr uint32_t kNone = 0xFFFFFFFFu;

__host__ __device__ constexpr uint32_t al16(uint32_t x) { return (x + 15u) & ~15u; }

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

struct RankTab {
    const uint4 *bucket;
    const uint32_t *pair;
    uint32_t nbk;
};

// Rank of the pair (a, b), or kNoRank. Specials and N never merge.
__device__ __forceinline__ uint32_t pair_rank(const RankTab &t, uint32_t a, uint32_t b) {
    if (a < 5 || a == 9 || b < 5 || b == 9) return kNoRank;
    const uint32_t key = a | (b << 16);
    uint32_t b1, b2;
    bpe_buckets(key, t.nbk, &b1, &b2);
    const uint4 x = t.bucket[b1], y = t.bucket[b2];
    uint32_t r = kNoRank;
    r = (x.x == key) ? x.y : r;
    r = (x.z == key) ? x.w : r;
    r = (y.x == key) ? y.y : r;
    r = (y.z == key) ? y.w : r;
    return r;
}

// Table layout in LDS: buckets, then 32-bit pairs.
__host__ __device__ inline uint32_t table_bytes(uint32_t nbk, int32_t R) {
    return 16u * nbk + al16(4u * (uint32_t)(R > 0 ? R : 1));
}

__device__ void load_table(uint8_t *dyn, const uint32_t *g_bucket, const uint32_t *g_pair, uint32_t nbk, int32_t R,
                           RankTab *t) {
    uint4 *bucket = reinterpret_cast<uint4 *>(dyn);
    uint32_t *pair = reinterpret_cast<uint32_t *>(dyn + 16u * nbk);
    const uint4 *gb = reinterpret_cast<const uint4 *>(g_bucket);
    for (uint32_t s = threadIdx.x; s < nbk; s += blockDim.x) bucket[s] = gb[s];
    for (int32_t r = threadIdx.x; r < R; r += blockDim.x) pair[r] = g_pair[r];
    *t = RankTab{bucket, pair, nbk};
}

// ---- 2. items ------------------------------------------------------------------

struct ItemArgs {
    const uint8_t *bytes;
    int64_t nbytes;
    const int64_t *offs;
    int32_t n;
    const int64_t *item_off;  // [n + 1]
    int64_t max_items;
    int32_t S;
    int64_t *item_start;
    int32_t *item_len;
    int32_t *item_cnt;
    int32_t ncls;         // length classes of the wave kernel
    int32_t cls_hi[4];    // class c takes lengths in (cls_hi[c-1], cls_hi[c]]
    uint32_t *qctl;       // [counts 4, tickets 4, done]
    int32_t *queue;       // [4][max_items] item indices per class
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

__global__ __launch_bounds__(NTE) void k_bpe_items(ItemArgs a) {
    const int lane = threadIdx.x & (dev::kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (NTE / dev::kWave);
    const int64_t total = min(a.item_off[a.n], a.max_items);
    for (int64_t t = (int64_t)blockIdx.x * (NTE / dev::kWave) + threadIdx.x / dev::kWave; t < total; t += waves) {
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
        if (lane == 0) {
            const int32_t len = (int32_t)(c1 > c0 ? c1 - c0 : 0);
            a.item_start[t] = c0;
            a.item_len[t] = len;
            a.item_cnt[t] = 0;
            // queue of its length class (longer items go to the workgroup kernel)
            int c = 0;
            while (c < a.ncls && len > a.cls_hi[c]) ++c;
            if (len > 0 && c < a.ncls) {
                const uint32_t pos = atomicAdd(a.qctl + c, 1u);
                a.queue[(int64_t)c * a.max_items + pos] = (int32_t)t;
            }
        }
    }
}

// ---- 3. wave per item ---------------------------------------------------------------

// Orders this wave's LDS accesses across lanes (a wave's LDS operations
// execute in order; the fences keep the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Minimum of the 64 pair ranks of block b (16-byte LDS reads).
__device__ __forceinline__ uint32_t block_min(const uint16_t *prk, uint32_t b) {
    const uint4 *src = reinterpret_cast<const uint4 *>(prk + (size_t)b * 64);
    uint32_t m = kNoRank;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const uint4 x = src[v];
        m = min(m, min(min(x.x & 0xFFFF, x.x >> 16), min(x.y & 0xFFFF, x.y >> 16)));
        m = min(m, min(min(x.z & 0xFFFF, x.z >> 16), min(x.w & 0xFFFF, x.w >> 16)));
    }
    return m;
}

struct WaveArgs {
    const uint8_t *bytes;
    const int64_t *item_start;
    const int32_t *item_len;
    int64_t max_items;
    uint16_t *tok;  // final symbols of item t at item_start[t]
    int32_t *item_cnt;
    const uint32_t *bucket;
    const uint32_t *pair;
    uint32_t nbk;
    int32_t R;
    // phases, longest items first: phase m runs mode_waves[m] waves per
    // workgroup, each holding up to mode_np[m] symbols, on queue mode_class[m]
    int32_t nmodes;
    int32_t mode_waves[4];
    uint32_t mode_np[4];
    uint32_t mode_wave_bytes[4];
    int32_t mode_class[4];
    uint32_t *qctl;  // [counts 4, tickets 4, done]
    const int32_t *queue;
    uint32_t *hdr;   // error word at hdr + 3
};

// A round merges the ranks present in a window [rs, rs + w) at once, w <= 64,
// as far as that equals merging them one after another; its occurrences sit
// in a list of at most kCap entries (kCap / 64 groups of a wave).
constexpr uint32_t kWin = 64;
constexpr uint32_t kCap = 256;
constexpr int kGroups = (int)(kCap / 64);

// Per-wave LDS, each part 16-byte aligned: sym[np], prk[np] (16-bit),
// alive[np/32], bmin[nb], cblk[nb] (16-bit), dirty[nb/32], and the round's
// occurrence list: list[kCap] and eq[kCap] (16-bit positions p and q),
// einfo[kCap] (8-bit: merges << 7 | rank - rs); nb = np / 64 blocks of 64
// positions, np a multiple of 64.
struct WaveLayout {
    uint32_t prk, alive, bmin, cblk, dirty, list, eq, einfo, bytes;
};
__host__ __device__ inline WaveLayout wave_layout(uint32_t np) {
    const uint32_t nb = np / 64;
    WaveLayout l;
    l.prk = 2u * np;
    l.alive = 4u * np;
    l.bmin = l.alive + al16(np / 8);
    l.cblk = l.bmin + al16(2u * nb);
    l.dirty = l.cblk + al16(2u * nb);
    l.list = l.dirty + al16(4u * ((nb + 31) / 32 + 1));
    l.eq = l.list + 2u * kCap;
    l.einfo = l.eq + 2u * kCap;
    l.bytes = l.einfo + kCap;
    return l;
}
__host__ __device__ inline uint32_t wave_lds_bytes(uint32_t np) { return wave_layout(np).bytes; }

// Alive positions around p from one 128-bit window of the bitmap (words
// w-1 .. w+2, w = p / 32): l = previous, q = next, q2 = the one after q.
// Positions outside the window are found by scanning words (rare: a dead
// run is shorter than the longest token). kNone where there is none.
struct Neighbors {
    uint32_t l, q, q2;
};

__device__ __forceinline__ uint32_t scan_up(const uint32_t *alive, uint32_t nw, uint32_t word) {
    for (; word < nw; ++word) {
        const uint32_t bits = alive[word];
        if (bits) return (word << 5) + (uint32_t)__builtin_ctz(bits);
    }
    return kNone;
}

__device__ __forceinline__ uint32_t scan_down(const uint32_t *alive, int32_t word) {
    for (; word >= 0; --word) {
        const uint32_t bits = alive[word];
        if (bits) return ((uint32_t)word << 5) + 31u - (uint32_t)__builtin_clz(bits);
    }
    return kNone;
}

// First set bit of the 128-bit (lo, hi) strictly above bit `rel`, or -1.
__device__ __forceinline__ int32_t window_next(uint64_t lo, uint64_t hi, int32_t rel) {
    if (rel < 63) {
        const uint64_t m = lo & (~0ull << (rel + 1));
        if (m) return __builtin_ctzll(m);
    }
    const int32_t rh = rel - 64;
    const uint64_t m2 = rh < 0 ? hi : (rh < 63 ? hi & (~0ull << (rh + 1)) : 0ull);
    return m2 ? 64 + __builtin_ctzll(m2) : -1;
}

__device__ __forceinline__ Neighbors neighbors(const uint32_t *alive, uint32_t nw, uint32_t p, bool want_q2) {
    const uint32_t w = p >> 5;
    const uint32_t a0 = w >= 1 ? alive[w - 1] : 0u;
    const uint32_t a1 = alive[w];
    const uint32_t a2 = w + 1 < nw ? alive[w + 1] : 0u;
    const uint32_t a3 = w + 2 < nw ? alive[w + 2] : 0u;
    const uint64_t lo = a0 | ((uint64_t)a1 << 32), hi = a2 | ((uint64_t)a3 << 32);
    const int32_t base = 32 * ((int32_t)w - 1);  // position of window bit 0
    const int32_t rel = 32 + (int32_t)(p & 31);
    Neighbors nb;
    const uint64_t below = lo & ((1ull << rel) - 1);
    nb.l = below ? (uint32_t)(base + 63 - __clzll(below)) : scan_down(alive, (int32_t)w - 2);
    const int32_t rq = window_next(lo, hi, rel);
    nb.q = rq >= 0 ? (uint32_t)(base + rq) : scan_up(alive, nw, w + 3);
    nb.q2 = kNone;
    if (want_q2 && nb.q != kNone) {
        if (rq >= 0) {
            const int32_t r2 = window_next(lo, hi, rq);
            nb.q2 = r2 >= 0 ? (uint32_t)(base + r2) : scan_up(alive, nw, w + 3);
        } else {
            // q itself lies beyond the window: continue from q
            const uint32_t wq = nb.q >> 5;
            const uint32_t bits = alive[wq] & ~((2u << (nb.q & 31)) - 1u);
            nb.q2 = bits ? (wq << 5) + (uint32_t)__builtin_ctz(bits) : scan_up(alive, nw, wq + 1);
        }
    }
    return nb;
}

constexpr int kK2Max = 16;  // level-2 blocks per lane (np <= 65536)

// One item, by one wave, in the LDS region at wb laid out for np symbols.
__device__ __forceinline__ void wave_item(const WaveArgs &a, const RankTab &tab, uint8_t *wb, uint32_t np, int64_t t) {
    const int lane = threadIdx.x & 63;
    const WaveLayout lay = wave_layout(np);
    uint16_t *sym = reinterpret_cast<uint16_t *>(wb);
    uint16_t *prk = reinterpret_cast<uint16_t *>(wb + lay.prk);
    uint32_t *alive = reinterpret_cast<uint32_t *>(wb + lay.alive);
    uint16_t *bmin = reinterpret_cast<uint16_t *>(wb + lay.bmin);
    uint16_t *cblk = reinterpret_cast<uint16_t *>(wb + lay.cblk);
    uint32_t *dirty = reinterpret_cast<uint32_t *>(wb + lay.dirty);
    uint16_t *list = reinterpret_cast<uint16_t *>(wb + lay.list);
    uint16_t *eq = reinterpret_cast<uint16_t *>(wb + lay.eq);
    uint8_t *einfo = wb + lay.einfo;
    const int32_t n = a.item_len[t];
    const int64_t c0 = a.item_start[t];
    const uint8_t *src = a.bytes + c0;
    const uint32_t nb = ((uint32_t)n + 63) / 64, nw = ((uint32_t)n + 31) / 32, k2 = (nb + 63) / 64;
    const uint32_t ndw = (nb + 31) / 32 + 1;  // dirty words (one spare: a lane's bits may straddle two)

    // symbols (four per lane per step), alive bits, dirty bits
    for (uint32_t p0 = 4 * lane; p0 < nb * 64; p0 += 256) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = p0 + u < (uint32_t)n ? symbol_of(src[p0 + u]) : 0u;
        *reinterpret_cast<uint2 *>(sym + p0) = make_uint2(v[0] | (v[1] << 16), v[2] | (v[3] << 16));
    }
    for (uint32_t w = lane; w < nb * 2; w += 64) {
        const int32_t f = n - 32 * (int32_t)w;
        alive[w] = f >= 32 ? ~0u : (f > 0 ? (1u << f) - 1u : 0u);
    }
    for (uint32_t w = lane; w < ndw; w += 64) dirty[w] = 0;
    wave_sync();
    // pair ranks and block minima, four blocks at a time
    for (uint32_t i = 0; i < nb; i += 4) {
        uint32_t r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t p = (i + u) * 64 + lane;
            const bool has = i + u < nb && p + 1 < (uint32_t)n;
            const uint32_t pn = has ? p + 1 : p;
            const uint32_t x = (i + u < nb) ? sym[p] : 0u, y = (i + u < nb) ? sym[pn] : 0u;
            r[u] = has ? pair_rank(tab, x, y) : kNoRank;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (i + u < nb) {
                prk[(i + u) * 64 + lane] = (uint16_t)r[u];
                const uint32_t m = dev::wave_min_all_u32(r[u]);
                if (lane == 0) bmin[i + u] = (uint16_t)m;
            }
        }
    }
    wave_sync();
    // level 2: this lane's blocks lane*k2 .. lane*k2 + k2 - 1, minima in registers
    const uint32_t b0 = (uint32_t)lane * k2;
    uint32_t bm[kK2Max];
    uint32_t l2 = kNoRank;
#pragma unroll
    for (int k = 0; k < kK2Max; ++k) {
        bm[k] = ((uint32_t)k < k2 && b0 + k < nb) ? (uint32_t)bmin[b0 + k] : kNoRank;
        l2 = min(l2, bm[k]);
    }

    // A round takes the lowest rank rs present and the ranks present just
    // above it, steps 0, 1, ... in rank order, and merges all their
    // occurrences at once where that gives what merging the ranks one after
    // another gives: occurrences of different ranks that share a symbol, or
    // a pair formed at a step before the last one whose rank is at most a
    // later step's rank, end the round's ranks before the later step
    // concerned. Every round merges rs, so rs strictly increases: at most R
    // rounds. When rs alone has more occurrences than the list holds, the
    // round takes them in chunks of whole blocks, each chunk gathered from
    // the state the previous one left (a merge's right element is gone from
    // it, and a pair between two chunks is rewritten from the later side).
    auto list_blocks = [&](uint32_t m) -> uint32_t {  // blocks of this lane's bits, in order, to cblk
        const uint32_t cc = (uint32_t)__popc(m);
        const uint32_t cinc = dev::wave_incl_sum_u32(cc);
        uint32_t o = cinc - cc;
        while (m) {
            cblk[o++] = (uint16_t)(b0 + (uint32_t)__builtin_ctz(m));
            m &= m - 1;
        }
        return dev::wave_read_u32(cinc, 63);
    };
    uint32_t Dn = kWin;
    for (int32_t round = 0;; ++round) {
        const uint32_t rs = dev::wave_min_all_u32(l2);
        if (rs == kNoRank) break;
        if (round > a.R) {
            if (lane == 0) dev::raise_error(a.hdr, DNATOK_DERR_INTERNAL);
            break;
        }
        // the window's occurrences in position order to the list, one block
        // per lane: a window of Dn ranks (what the last rounds' lists
        // suggest), narrowed fourfold while its occurrences overflow the list
        const uint32_t w64 = min(kWin, (uint32_t)kNoRank - rs);
        auto block_window = [&](uint32_t b, uint32_t w) -> uint64_t {  // positions of block b ranked in [rs, rs + w)
            const uint4 *src = reinterpret_cast<const uint4 *>(prk + (size_t)b * 64);
            uint64_t m = 0;
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const uint4 x = src[v];
                const uint32_t wd[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    m |= (uint64_t)((wd[u] & 0xFFFFu) - rs < w) << (8 * v + 2 * u);
                    m |= (uint64_t)((wd[u] >> 16) - rs < w) << (8 * v + 2 * u + 1);
                }
            }
            return m;
        };
        // a single rank whose occurrences overflow the list goes in chunks of whole blocks
        bool dense = false;
        uint32_t D = 0, total = 0, Dc = min(Dn, w64), own_dirty = 0, ncb = 0;
        for (;;) {
            uint32_t cm = 0;
#pragma unroll
            for (int k = 0; k < kK2Max; ++k) cm |= (uint32_t)(bm[k] - rs < Dc) << k;
            ncb = list_blocks(cm);
            wave_sync();
            uint32_t cnt = 0;
            for (uint32_t j0 = 0; j0 < ncb; j0 += 64) {
                const uint32_t j = j0 + (uint32_t)lane;
                const uint32_t b = j < ncb ? (uint32_t)cblk[j] : 0u;
                uint64_t m = j < ncb ? block_window(b, Dc) : 0ull;
                const uint32_t c = (uint32_t)__popcll(m);
                const uint32_t inc = dev::wave_incl_sum_u32(c);
                for (uint32_t o = cnt + inc - c; m && o < kCap; ++o, m &= m - 1)
                    list[o] = (uint16_t)(b * 64 + (uint32_t)__builtin_ctzll(m));
                cnt += dev::wave_read_u32(inc, 63);
            }
            if (cnt <= kCap) {
                D = Dc;
                total = cnt;
                own_dirty = cm;  // these blocks are all refreshed after the round
                break;
            }
            if (Dc == 1) {
                dense = true;
                D = 1;
                own_dirty = cm;
                break;
            }
            Dc = max(1u, Dc / 4);
            wave_sync();
        }
        // the next round's window: wider after a short list, narrower after a long one
        if (dense)
            Dn = 1;
        else if (3 * total <= kCap)
            Dn = min(kWin, 2 * D);
        else if (3 * total > 2 * kCap)
            Dn = max(1u, D / 2);
        else
            Dn = D;
        uint32_t jb = 0;  // dense: the next candidate block
        do {
            if (dense) {
                // blocks from jb on, whole blocks while their occurrences fit the list
                wave_sync();
                const uint32_t j = jb + (uint32_t)lane;
                const uint32_t b = j < ncb ? (uint32_t)cblk[j] : 0u;
                uint64_t m = j < ncb ? block_window(b, 1u) : 0ull;
                const uint32_t c = (uint32_t)__popcll(m);
                const uint32_t inc = dev::wave_incl_sum_u32(c);
                const bool take = j < ncb && inc <= kCap;  // a prefix of the lanes, at least one
                const uint32_t ntake = (uint32_t)__popcll(__ballot(take));
                if (take)
                    for (uint32_t o = inc - c; m; ++o, m &= m - 1)
                        list[o] = (uint16_t)(b * 64 + (uint32_t)__builtin_ctzll(m));
                total = ntake ? dev::wave_read_u32(inc, ntake - 1) : 0u;
                jb += ntake;
            }
            wave_sync();
            // pass 1, per occurrence: its neighbours, and whether it merges
            // (all occurrences of a rank, or for (X, X) every other one of a
            // run, leftmost first); q and the outcome go to the list
            uint32_t Pg[kGroups], Qg[kGroups], Lg[kGroups], Q2g[kGroups], Dg[kGroups];
            bool Mg[kGroups];
            uint64_t pres_l = 0;
            uint32_t carry_q = kNone, carry_d = kNone;
            int32_t carry_off = 0;
#pragma unroll
            for (int g = 0; g < kGroups; ++g) {
                Pg[g] = 0;
                Qg[g] = Lg[g] = Q2g[g] = kNone;
                Dg[g] = 0;
                Mg[g] = false;
                if ((uint32_t)(64 * g) < total) {
                    const uint32_t e = 64u * g + (uint32_t)lane;
                    const bool valid = e < total;
                    const uint32_t p = valid ? (uint32_t)list[e] : 0u;
                    const uint32_t r = valid ? (uint32_t)prk[p] : (uint32_t)kNoRank;
                    const uint32_t d = r - rs;
                    Neighbors nbr{kNone, kNone, kNone};
                    if (valid) nbr = neighbors(alive, nw, p, true);
                    const uint32_t pr = valid ? tab.pair[r] : 0u;
                    const bool chain = valid && (pr & 0xFFFFu) == (pr >> 16);
                    const uint32_t q_up = dev::wave_from_prev_u32(nbr.q, carry_q);
                    const uint32_t d_up = dev::wave_from_prev_u32(d, carry_d);
                    const bool adj = chain && q_up == p && d_up == d;
                    const uint64_t starts = __ballot(valid && !adj);
                    const uint64_t below = starts & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
                    const int32_t off = below ? lane - (63 - __clzll(below)) : carry_off + 1 + lane;
                    const bool ms = valid && (!chain || (off & 1) == 0);
                    const uint32_t last = min(total - 64u * g, 64u) - 1u;
                    carry_q = dev::wave_read_u32(nbr.q, last);
                    carry_d = dev::wave_read_u32(d, last);
                    carry_off = (int32_t)dev::wave_read_u32((uint32_t)off, last);
                    if (valid) {
                        eq[e] = (uint16_t)nbr.q;
                        einfo[e] = (uint8_t)((ms ? 0x80u : 0u) | d);
                        pres_l |= 1ull << d;
                    }
                    Pg[g] = p;
                    Qg[g] = nbr.q;
                    Lg[g] = nbr.l;
                    Q2g[g] = nbr.q2;
                    Dg[g] = d;
                    Mg[g] = ms;
                }
            }
            // ranks present: step of rank rs + d = ranks present below it
            const uint64_t pres = ((uint64_t)dev::wave_or_all_u32((uint32_t)(pres_l >> 32)) << 32) |
                                  dev::wave_or_all_u32((uint32_t)pres_l);
            const uint32_t nsteps = (uint32_t)__popcll(pres);
            auto step_of = [&](uint32_t d) { return (uint32_t)__popcll(pres & ((1ull << d) - 1ull)); };
            // a pair of rank r formed at step st allows steps up to this bound (exclusive)
            auto bound = [&](uint32_t st, uint32_t r) -> uint32_t {
                if (r == kNoRank) return nsteps;
                const uint32_t idx = r < rs ? 0u : (r - rs >= 64u ? nsteps : step_of(r - rs));
                return max(st + 1u, idx);
            };
            wave_sync();
            // pass 2, per merging occurrence: the pairs it forms on each side,
            // at its own step and, next to a merge of another step, at the
            // later of the two; the bound they and shared symbols set
            uint32_t Ag[kGroups], RFg[kGroups], RIg[kGroups], LIg[kGroups], BRg[kGroups], BLg[kGroups];
            uint32_t cutv = nsteps;
#pragma unroll
            for (int g = 0; g < kGroups; ++g) {
                Ag[g] = 0;
                RFg[g] = RIg[g] = LIg[g] = kNoRank;
                BRg[g] = BLg[g] = kNone;
                if ((uint32_t)(64 * g) < total) {
                    // every read an entry may need goes out at once (indices
                    // clamped, results selected after), then the three
                    // lookups: branches per case kept the LDS trips apart
                    const uint32_t e = 64u * g + (uint32_t)lane;
                    const bool ms = Mg[g];
                    const uint32_t d = Dg[g], st = step_of(d), NEW = 10u + rs + d;
                    const uint32_t q2 = Q2g[g], l = Lg[g];
                    const uint32_t e1 = min(e + 1, kCap - 1), e2 = min(e + 2, kCap - 1);
                    const uint32_t m1 = e >= 1 ? e - 1 : 0u, m2 = e >= 2 ? e - 2 : 0u;
                    const uint32_t p1 = list[e1], p2 = list[e2], i1 = einfo[e1], i2 = einfo[e2];
                    const uint32_t qm1 = eq[m1], qm2 = eq[m2], im1 = einfo[m1], im2 = einfo[m2];
                    const uint32_t s2 = sym[q2 != kNone ? q2 : 0u], sl = sym[l != kNone ? l : 0u];
                    // a merge starting at q2, one or two entries on
                    const bool r1 = q2 != kNone && e + 1 < total && p1 == q2 && (i1 & 0x80u);
                    const bool r2 = !r1 && q2 != kNone && e + 2 < total && p2 == q2 && (i2 & 0x80u);
                    const bool jr = r1 || r2;
                    const uint32_t dj = (r1 ? i1 : i2) & 63u, sj = step_of(dj);
                    // a merge ending at l, one or two entries back
                    const bool l1 = l != kNone && e >= 1 && qm1 == l && (im1 & 0x80u);
                    const bool l2b = !l1 && l != kNone && e >= 2 && qm2 == l && (im2 & 0x80u);
                    const bool jl = l1 || l2b;
                    const uint32_t sl_step = step_of((l1 ? im1 : im2) & 63u);
                    // the pairs this merge forms: with the merge on the right
                    // (at the later step), and with the unmerged symbol on
                    // each side (at its own step)
                    const uint32_t rf = pair_rank(tab, NEW, 10u + rs + dj);
                    const uint32_t ri = pair_rank(tab, NEW, s2);
                    const uint32_t li = pair_rank(tab, sl, NEW);
                    const bool need_ri = q2 != kNone && (!jr || sj > st);
                    const bool need_li = l != kNone && (!jl || sl_step > st);
                    if (ms) {
                        Ag[g] = st;
                        if (jr) {
                            BRg[g] = sj;
                            RFg[g] = rf;
                            cutv = min(cutv, bound(max(st, sj), rf));
                        }
                        if (need_ri) {
                            RIg[g] = ri;
                            cutv = min(cutv, bound(st, ri));
                        }
                        if (jl) BLg[g] = sl_step;
                        if (need_li) {
                            LIg[g] = li;
                            cutv = min(cutv, bound(st, li));
                        }
                        // the previous entry merges too and shares p: another step ends before the later one
                        if (e >= 1 && (im1 & 0x80u) && qm1 == Pg[g] && (im1 & 63u) != d)
                            cutv = min(cutv, max(st, step_of(im1 & 63u)));
                    }
                }
            }
            const uint32_t cut = dev::wave_min_all_u32(cutv);
            wave_sync();
            // pass 3: the merges of steps below the bound; a side whose
            // neighbouring merge also happens is written by the left one
#pragma unroll
            for (int g = 0; g < kGroups; ++g) {
                if ((uint32_t)(64 * g) < total && Mg[g] && Ag[g] < cut) {
                    const uint32_t p = Pg[g], q = Qg[g], l = Lg[g], st = Ag[g];
                    sym[p] = (uint16_t)(10u + rs + Dg[g]);
                    prk[p] = (uint16_t)((BRg[g] != kNone && BRg[g] < cut) ? RFg[g] : RIg[g]);
                    prk[q] = kNoRank;
                    atomicAnd(&alive[q >> 5], ~(1u << (q & 31)));
                    // p's block is refreshed; q's and l's may be neighbours
                    if ((q >> 6) != (p >> 6)) atomicOr(&dirty[(q >> 6) >> 5], 1u << ((q >> 6) & 31));
                    if (l != kNone && (BLg[g] == kNone || (BLg[g] > st && BLg[g] >= cut))) {
                        prk[l] = (uint16_t)LIg[g];
                        if ((l >> 6) != (p >> 6)) atomicOr(&dirty[(l >> 6) >> 5], 1u << ((l >> 6) & 31));
                    }
                }
            }
            wave_sync();
        } while (dense && jb < ncb);
        // refresh the minima of this lane's changed blocks
        {
            const uint32_t w0 = b0 >> 5;
            const uint64_t dw = b0 < nb ? ((uint64_t)dirty[w0] | ((uint64_t)dirty[w0 + 1] << 32)) : 0ull;
            own_dirty |= (uint32_t)(dw >> (b0 & 31)) & ((k2 >= 32) ? ~0u : ((1u << k2) - 1u));
        }
        // the changed blocks listed, one per lane recomputed into bmin (a
        // pass per lane's own changed block made the wave wait for its
        // busiest lane: 3,800 cycles per round), then each lane's minima
        // read back
        wave_sync();
        const uint32_t nch = list_blocks(own_dirty);
        wave_sync();
        for (uint32_t j = (uint32_t)lane; j < nch; j += 64) {
            const uint32_t b = cblk[j];
            bmin[b] = (uint16_t)block_min(prk, b);
        }
        wave_sync();
        if (own_dirty) {
#pragma unroll
            for (int k = 0; k < kK2Max; ++k)
                if ((own_dirty >> k) & 1u) bm[k] = bmin[b0 + (uint32_t)k];
            l2 = kNoRank;
#pragma unroll
            for (int k = 0; k < kK2Max; ++k) l2 = min(l2, bm[k]);
        }
        wave_sync();
        for (uint32_t w = lane; w < ndw; w += 64) dirty[w] = 0;
        wave_sync();
    }

    // surviving symbols in order
    uint32_t cnt = 0;
    uint16_t *out = a.tok + c0;
    for (uint32_t base = 0; base < nb * 64; base += 64) {
        const uint32_t p = base + lane;
        const bool on = (alive[p >> 5] >> (p & 31)) & 1u;
        const uint64_t mk = __ballot(on);
        if (on) out[cnt + (uint32_t)__popcll(mk & ((1ull << lane) - 1))] = sym[p];
        cnt += (uint32_t)__popcll(mk);
    }
    if (lane == 0) a.item_cnt[t] = (int32_t)cnt;
    wave_sync();
}

// Persistent BPE over all length classes in one launch: every workgroup
// takes the longest class first (one wave with the whole LDS), then shorter
// classes with more waves sharing it, pulling items from each class's queue;
// a workgroup barrier separates the phases because the LDS is re-divided.
__global__ __launch_bounds__(kMaxWaves * 64) void k_bpe_wave(WaveArgs a) {
    extern __shared__ __align__(16) uint8_t dyn[];
    RankTab tab;
    load_table(dyn, a.bucket, a.pair, a.nbk, a.R, &tab);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x / 64;
    uint8_t *pool = dyn + table_bytes(a.nbk, a.R);
    for (int m = 0; m < a.nmodes; ++m) {
        if (wave < a.mode_waves[m]) {
            const int c = a.mode_class[m];
            const uint32_t count = a.qctl[c];
            uint8_t *wb = pool + (size_t)wave * a.mode_wave_bytes[m];
            for (;;) {
                uint32_t tk = 0;
                if (lane == 0) tk = atomicAdd(a.qctl + 4 + c, 1u);
                tk = dev::wave_read_u32(tk, 0);
                if (tk >= count) break;
                wave_item(a, tab, wb, a.mode_np[m], (int64_t)a.queue[(int64_t)c * a.max_items + tk]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // the last workgroup to finish empties the queues for the next launch
        if (atomicAdd(a.qctl + 8, 1u) == gridDim.x - 1)
            for (int i = 0; i < 9; ++i) dev::st_relaxed32(a.qctl + i, 0u);
    }
}

// ---- 4. workgroup per long item ---------------------------------------------------

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
    Chain lw;
    lw.full = __shfl_up(inc.full, 1, dev::kWave);
    lw.tail = __shfl_up(inc.tail, 1, dev::kWave);
    lw.len = __shfl_up(inc.len, 1, dev::kWave);
    __syncthreads();
    return lane == 0 ? pre : chain_join(pre, lw);
}

// Segment A[0, n) with B as the second buffer (global scratch). A rank
// histogram of all current pairs drives the rounds; each round merges,
// compacts into the other buffer and updates the histogram for the pairs
// destroyed and created. Returns the final length; *in_a tells whether the
// result ended up in A.
__device__ int32_t merge_segment(uint16_t *A, uint16_t *B, int32_t n, const RankTab &tab, int32_t *hist, int32_t R,
                                 int64_t *s_tmp, Chain *s_chain, int32_t *s_rstar, bool *in_a) {
    const int tid = threadIdx.x;
    const int lane = tid & (dev::kWave - 1);
    bool a_is_a = true;
    for (int32_t r = tid; r < R; r += NTM) hist[r] = 0;
    __syncthreads();
    for (int32_t p = tid; p + 1 < n; p += NTM) {
        const uint32_t r = pair_rank(tab, A[p], A[p + 1]);
        if (r != kNoRank) atomicAdd(&hist[r], 1);
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
        const uint32_t pr = tab.pair[rs];
        const uint16_t L = (uint16_t)(pr & 0xFFFF), Rr = (uint16_t)(pr >> 16);
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
                        const uint32_t r2 = pair_rank(tab, Rr, A[p + 2]);
                        if (r2 != kNoRank) atomicSub(&hist[r2], 1);
                    }
                    // the left pair belongs to this merge unless p-1 was consumed by a merge at p-2
                    const bool p2 = (p >= 2) && cand(p - 2) && (!chain || cand(p - 1));
                    if (p >= 1 && !p2) {
                        const uint32_t r0 = pair_rank(tab, A[p - 1], L);
                        if (r0 != kNoRank) atomicSub(&hist[r0], 1);
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
                            const uint32_t r = pair_rank(tab, NEW, B[y + 1]);
                            if (r != kNoRank) atomicAdd(&hist[r], 1);
                        }
                        if (y >= 1 && B[y - 1] != NEW) {
                            const uint32_t r = pair_rank(tab, B[y - 1], NEW);
                            if (r != kNoRank) atomicAdd(&hist[r], 1);
                        }
                    }
                    ++y;
                }
                prev = ms;
            }
        }
        __syncthreads();
        uint16_t *t = A;
        A = B;
        B = t;
        a_is_a = !a_is_a;
        n = (int32_t)n2;
    }
    *in_a = a_is_a;
    return n;
}

struct BlockArgs {
    const uint8_t *bytes;
    const int64_t *item_start;
    const int32_t *item_len;
    const int64_t *n_items_at;
    int64_t max_items;
    uint16_t *symA;  // [nbytes]: final symbols of every item at its start
    uint16_t *symB;  // [nbytes]: second buffer
    int32_t *item_cnt;
    const uint32_t *bucket;
    const uint32_t *pair;
    uint32_t nbk;
    int32_t R;
    int32_t lo;  // this launch takes items longer than lo
    uint32_t *hdr;
};

__global__ __launch_bounds__(NTM) void k_bpe_block(BlockArgs a) {
    extern __shared__ __align__(16) uint8_t dyn[];
    __shared__ int64_t s_tmp[NTM / dev::kWave + 1];
    __shared__ Chain s_chain[NTM / dev::kWave];
    __shared__ int32_t s_rstar;
    __shared__ int64_t s_ticket;
    RankTab tab;
    load_table(dyn, a.bucket, a.pair, a.nbk, a.R, &tab);
    int32_t *hist = reinterpret_cast<int32_t *>(dyn + table_bytes(a.nbk, a.R));
    const int tid = threadIdx.x;
    const int64_t total = min(*a.n_items_at, a.max_items);
    __syncthreads();
    for (;;) {
        if (tid == 0) s_ticket = (int64_t)atomicAdd(a.hdr + 0, 1u);
        __syncthreads();
        const int64_t t = s_ticket;
        __syncthreads();
        if (t >= total) break;
        const int32_t len = a.item_len[t];
        if (len <= a.lo) continue;
        const int64_t c0 = a.item_start[t];
        uint16_t *ga = a.symA + c0, *gb = a.symB + c0;
        for (int32_t p = tid; p < len; p += NTM) ga[p] = symbol_of(a.bytes[c0 + p]);
        __syncthreads();
        bool in_a = true;
        const int32_t nf = merge_segment(ga, gb, len, tab, hist, a.R, s_tmp, s_chain, &s_rstar, &in_a);
        if (!in_a)
            for (int32_t p = tid; p < nf; p += NTM) ga[p] = gb[p];
        if (tid == 0) a.item_cnt[t] = nf;
        __syncthreads();
    }
    if (tid == 0) dev::finish_block(a.hdr, false);
}

// ---- 5. item count scan and emit ---------------------------------------------------

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
            // unconditional load of a clamped entry (an empty batch, total
            // 0, loads nothing), so the thread's loads go out together
            const int64_t x = total > 0 ? a.cnt[i0 + j < total ? i0 + j : total - 1] : 0;
            v[j] = (i0 + j < total) ? x : 0;
            mine += v[j];
        }
        int64_t utot;
        const int64_t pre = dev::block_excl_scan<NTE>(mine, s_tmp, &utot);
        if (tid < dev::kWave) {
            if (tid == 0) dev::publish_aggregate(st, u, utot);
            const int64_t ex = dev::wave_lookback(st, u, utot, a.q.hdr);
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

// Length classes of the wave kernel for a table of `tab` LDS bytes: waves
// per workgroup w in {8, 4, 2, 1} (those <= max_waves), each wave holding up
// to np(w) symbols
// where one workgroup fills the CU's LDS. Class w takes the items longer
// than the previous class's capacity.
int bpe_wave_classes(uint32_t tab, int max_waves, BpeClass *out, int max_out) {
    int nc = 0;
    uint32_t prev = 0;
    const int waves[4] = {8, 4, 2, 1};
    for (int i = 0; i < 4 && nc < max_out; ++i) {
        const int w = waves[i];
        if (w > max_waves) continue;
        if (kLdsBytes < kLdsReserve + tab) break;
        const size_t room = (kLdsBytes - kLdsReserve - tab) / (size_t)w;
        // largest multiple of 64 whose per-wave layout fits the room
        uint32_t np = (uint32_t)std::min<size_t>(room / 4, 65536) / 64 * 64;
        while (np >= 64 && wave_lds_bytes(np) > room) np -= 64;
        if (np < 64 || np <= prev) continue;
        out[nc].waves = w;
        out[nc].lo = (int32_t)prev;
        out[nc].hi = (int32_t)np;
        out[nc].np = np;
        out[nc].lds = tab + (uint32_t)w * wave_lds_bytes(np);
        prev = np;
        ++nc;
    }
    return nc;
}

namespace {
// Scratch of one BPE encode: symA, symB (uint16 per byte), item offsets,
// counts, lengths, starts, positions and the four length-class queues.
struct BpeScratch {
    int64_t max_items, sz_sym, sz_ioff, sz_cnt, sz_start, sz_pos, sz_queue, total;
};
BpeScratch bpe_scratch(int64_t nbytes, int32_t n, int32_t S) {
    auto al = [](int64_t x) { return (x + 255) / 256 * 256; };
    BpeScratch b;
    b.max_items = nbytes / S + (int64_t)n + 1;
    b.sz_sym = al(2 * (nbytes + 1));
    b.sz_ioff = al(8 * ((int64_t)n + 1));
    b.sz_cnt = al(4 * b.max_items);
    b.sz_start = al(8 * b.max_items);
    b.sz_pos = al(8 * (b.max_items + 1));
    b.sz_queue = al(4 * 4 * b.max_items);
    b.total = 2 * b.sz_sym + b.sz_ioff + 2 * b.sz_cnt + b.sz_start + b.sz_pos + b.sz_queue;
    return b;
}
}  // namespace

int64_t bpe_scratch_bytes(int64_t nbytes, int32_t n, int32_t S) { return bpe_scratch(nbytes, n, S).total; }

int64_t bpe_workspace_tiles(int64_t nbytes, int32_t n, int32_t S) {
    const int64_t units_rows = std::max<int64_t>(1, ((int64_t)n + 4095) / 4096);
    const int64_t units_items =
        std::max<int64_t>(1, (bpe_scratch(nbytes, n, S).max_items + kScanUnit - 1) / kScanUnit);
    return std::max(units_rows, units_items);
}

int launch_bpe_encode(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                      int32_t n, int32_t *d_ids, int64_t cap, int64_t *d_out_offsets, int8_t *d_mask,
                      const dnatok_encode_opts &o, hipStream_t stream) {
    const BpeTables &bt = v->bpe;
    const int32_t R = bt.n_merges;
    const int32_t ti = v->tune_item.load(std::memory_order_relaxed);
    const int32_t S = ti > 0 ? ti : kBpeItemBytesDefault;
    const int32_t tw = v->tune_waves.load(std::memory_order_relaxed);
    const int max_waves = tw > 0 ? tw : kMaxWaves;
    const BpeScratch bs = bpe_scratch(nbytes, n, S);
    const int64_t max_items = bs.max_items;
    const int64_t sz_sym = bs.sz_sym, sz_ioff = bs.sz_ioff, sz_cnt = bs.sz_cnt, sz_start = bs.sz_start;
    Workspace *ws = nullptr;
    const int64_t units_items = std::max<int64_t>(1, (max_items + kScanUnit - 1) / kScanUnit);
    int rc = get_workspace(stream, bpe_workspace_tiles(nbytes, n, S), &ws);
    if (rc) return rc;
    rc = ensure_scratch(ws, bs.total);
    if (rc) return rc;
    uint8_t *sp = ws->d_scratch;
    uint16_t *symA = reinterpret_cast<uint16_t *>(sp);
    sp += sz_sym;
    uint16_t *symB = reinterpret_cast<uint16_t *>(sp);
    sp += sz_sym;
    int64_t *item_off = reinterpret_cast<int64_t *>(sp);
    sp += sz_ioff;
    int32_t *item_cnt = reinterpret_cast<int32_t *>(sp);
    sp += sz_cnt;
    int32_t *item_len = reinterpret_cast<int32_t *>(sp);
    sp += sz_cnt;
    int64_t *item_start = reinterpret_cast<int64_t *>(sp);
    sp += sz_start;
    int64_t *item_pos = reinterpret_cast<int64_t *>(sp);
    sp += bs.sz_pos;
    int32_t *queue = reinterpret_cast<int32_t *>(sp);
    if (units_items > ws->high_water) ws->high_water = units_items;
    const int cus = device_cu_count();

    // 1. item plan
    rc = launch_rowscan(d_offsets, n, nbytes, item_off, S, 0, stream);
    if (rc) return rc;

    // 2. items
    const uint32_t tab = table_bytes(bt.nbk, R);
    BpeClass cls[4];
    const int ncls = bpe_wave_classes(tab, max_waves, cls, 4);
    uint32_t *qctl = ws->d_hdr + HDR_BPE_QUEUES;  // self-resetting queue counters
    ItemArgs ia{d_bytes, nbytes, d_offsets, n, item_off, max_items, S, item_start, item_len, item_cnt,
                ncls, {0, 0, 0, 0}, qctl, queue};
    for (int c = 0; c < ncls; ++c) ia.cls_hi[c] = cls[c].hi;
    const int64_t g_items = std::max<int64_t>(1, std::min<int64_t>((max_items + 3) / 4, (int64_t)cus * 8));
    hipLaunchKernelGGL(k_bpe_items, dim3((unsigned)g_items), dim3(NTE), 0, stream, ia);
    DNATOK_HIP(hipGetLastError());

    // 3. all length classes in one persistent launch, longest first
    int32_t covered = 0;
    if (ncls > 0) {
        WaveArgs w;
        w.bytes = d_bytes;
        w.item_start = item_start;
        w.item_len = item_len;
        w.max_items = max_items;
        w.tok = symA;
        w.item_cnt = item_cnt;
        w.bucket = bt.d_bucket;
        w.pair = bt.d_pair;
        w.nbk = bt.nbk;
        w.R = R;
        w.nmodes = ncls;
        uint32_t lds = 0;
        int wmax = 1;
        for (int m = 0; m < ncls; ++m) {
            const BpeClass &c = cls[ncls - 1 - m];
            w.mode_waves[m] = c.waves;
            w.mode_np[m] = c.np;
            w.mode_wave_bytes[m] = wave_lds_bytes(c.np);
            w.mode_class[m] = ncls - 1 - m;
            lds = std::max(lds, c.lds);
            wmax = std::max(wmax, c.waves);
        }
        w.qctl = qctl;
        w.queue = queue;
        w.hdr = ws->d_hdr;
        DNATOK_HIP(hipFuncSetAttribute((const void *)k_bpe_wave, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds));
        hipLaunchKernelGGL(k_bpe_wave, dim3((unsigned)cus), dim3(64 * wmax), lds, stream, w);
        DNATOK_HIP(hipGetLastError());
        covered = cls[ncls - 1].hi;
    }

    // 4. longer items
    {
        BlockArgs b;
        b.bytes = d_bytes;
        b.item_start = item_start;
        b.item_len = item_len;
        b.n_items_at = item_off + n;
        b.max_items = max_items;
        b.symA = symA;
        b.symB = symB;
        b.item_cnt = item_cnt;
        b.bucket = bt.d_bucket;
        b.pair = bt.d_pair;
        b.nbk = bt.nbk;
        b.R = R;
        b.lo = covered;
        b.hdr = ws->d_hdr;
        const size_t dyn = tab + 4 * (size_t)(R > 0 ? R : 1);
        DNATOK_HIP(hipFuncSetAttribute((const void *)k_bpe_block, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)dyn));
        hipLaunchKernelGGL(k_bpe_block, dim3((unsigned)cus), dim3(NTM), dyn, stream, b);
        DNATOK_HIP(hipGetLastError());
    }

    // 5. item positions and output
    ScanArgs sa;
    sa.cnt = item_cnt;
    sa.total_at = item_off + n;
    sa.pos = item_pos;
    sa.max_items = max_items;
    sa.nunits = units_items;
    sa.q.hdr = ws->d_hdr;
    sa.q.status0 = ws->d_status;
    sa.q.status1 = ws->d_status + ws->cap;
    sa.q.clear_n = ws->high_water;
    int per_cu = 0;
    DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_scan_counts, NTE, 0));
    int64_t g2 = std::min<int64_t>(units_items, (int64_t)cus * std::max(per_cu, 1));
    hipLaunchKernelGGL(k_scan_counts, dim3((unsigned)g2), dim3(NTE), 0, stream, sa);
    DNATOK_HIP(hipGetLastError());

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
    int64_t g3 = std::max<int64_t>(1, std::min<int64_t>(std::max<int64_t>(n, max_items), (int64_t)cus * 8));
    hipLaunchKernelGGL(k_bpe_emit, dim3((unsigned)g3), dim3(NTE), 0, stream, e);
    DNATOK_HIP(hipGetLastError());
    return DNATOK_OK;
}

}  // namespace dnatok
