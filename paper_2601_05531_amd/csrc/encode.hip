// Byte -> identifier encode of a ragged batch (SINGLE, LUT256, KMER).
//
// Paper: Design, "Encoding paths", bytes path (a device-resident 256-entry
// LUT applied to staged ASCII) and the bytes branch of the EmbedFromStrings
// algorithm (MapKmer for k-mer vocabularies, left padding to token_len).
//
// MI355X-first decomposition (the paper applies ascii_lut[Bytes] as a
// framework tensor op on an equal-length B x T matrix):
//  * Row scan (k_rowscan): every row's token count has a closed form
//    (L, or ceil(L/k), plus 2 with CLS/SEP), so out_offsets is a scan over
//    rows. Units of 4096 rows are handed out by ticket and chained with a
//    decoupled look-back; a batch of a few thousand rows is one unit.
//  * Cell kernel (k_cells): the concatenated input is cut into fixed tiles
//    of B bytes, addressed from the 16-byte-aligned base so every tile load
//    is a full 16-byte vector load. Every output cell is owned by the tile
//    holding its anchor byte: CLS at the row start, body token j at
//    off + j*k, SEP at the row's last byte, pads at the CLS (left) or SEP
//    (right) anchor. A tile therefore owns one contiguous run of cells per
//    row it touches and its work is bounded by B whatever the row lengths.
//    Cell positions follow from out_offsets (PACKED) or row * width
//    (PADDED), so tiles never wait on each other: blocks walk a static
//    grid-stride tile sequence with no atomics at all.
//  * Each tile is staged into LDS once with coalesced 16-byte loads; the
//    next tile's loads are issued before the current tile is written.
//    k-mer tiles are classified on the way in: 2-bit base digits packed
//    most-significant-first (16 bases per word) plus one validity bit per
//    base, so a k-mer id is two funnel shifts and a mask compare.
//    Single-base tiles keep raw bytes, with the 256-entry table in LDS.
//  * Stores go out as aligned 16-byte groups of four ids (plus one 4-byte
//    mask word in PADDED layout); ragged group edges use scalar stores.
//  * PADDED layout with a modest row count fuses the row scan into one
//    extra block of the cell kernel: a single launch.
#include "common.hpp"
#include "device.hpp"

namespace dnatok {

namespace {

constexpr int NT = 256;
constexpr int kRowsPerThread = 16;                   // row scan: rows per thread per pass
constexpr int64_t kUnitRows = (int64_t)NT * kRowsPerThread;
constexpr int32_t kFuseMaxRows = 16384;              // PADDED: fold the row scan into the cell launch
constexpr int kMaxMultiVocabs = 8;                    // vocabularies one cell launch can write
constexpr int32_t kFusePackedRows = 2 * NT;            // PACKED, one vocabulary: every block scans the rows itself
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

// Number of body tokens of a row of L bytes.
__device__ __forceinline__ int64_t body_tokens(int64_t L, int32_t k, bool kmer) {
    if (!kmer) return L;
    const int64_t span = L + k - 1;
    return span < 0x7FFFFFFF ? (int64_t)((uint32_t)span / (uint32_t)k) : span / k;
}

struct Row {
    int64_t off, end, nb, len;
};

// Tokens of the row whose anchor byte is < X.
__device__ __forceinline__ int64_t tokens_before(const Row &r, int64_t X, int32_t k, int32_t cls) {
    int64_t c = 0;
    if (X > r.off) {
        // body anchors off + j*k < X  <=>  j < ceil((X - off) / k)
        const int64_t span = X - r.off + k - 1;
        c += (X >= r.end) ? r.nb : (span < 0x7FFFFFFF ? (int64_t)((uint32_t)span / (uint32_t)k) : span / k);
        if (cls) c += 1;  // CLS anchored at off
    }
    if (cls) {
        int64_t sep_anchor = (r.end > r.off) ? r.end - 1 : r.off;
        if (sep_anchor < X) c += 1;
    }
    return c;
}

// Cells (tokens plus pads) of the row whose anchor is < X.
__device__ __forceinline__ int64_t cells_before(const Row &r, int64_t X, int32_t k, int32_t cls, int32_t padded,
                                                int32_t left, int64_t W) {
    int64_t c = tokens_before(r, X, k, cls);
    if (!padded) return c;
    int64_t pads = W - r.len;
    if (left) {
        if (r.off < X) c += pads;
    } else {
        int64_t last_anchor;
        if (r.len == 0) last_anchor = r.off;
        else if (cls) last_anchor = (r.end > r.off) ? r.end - 1 : r.off;
        else last_anchor = r.off + (r.nb - 1) * k;
        if (last_anchor < X) c += pads;
    }
    return c;
}

// 16 bytes -> 16 two-bit base digits (most significant first) and 16
// validity bits (bit 31 = first byte) for the A/C/G/T/a/c/g/t test. Per 4
// bytes: fold case, read the digit off bits 1-2 (a->0 c->1 g->2 t->3), look
// the canonical letter of that digit up with a byte permute, and compare;
// multiplies gather the 2-bit digits and the validity bits.
__device__ __forceinline__ void classify16(uint4 v, uint32_t &code, uint32_t &valid) {
    const uint32_t x[4] = {v.x, v.y, v.z, v.w};
    code = 0;
    valid = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t f = x[q] | 0x20202020u;  // only A/a map to a (likewise c, g, t)
        const uint32_t d = ((f >> 1) ^ (f >> 2)) & 0x03030303u;
        const uint32_t canon = __builtin_amdgcn_perm(0u, 0x74676361u, d);  // "acgt"[d] per byte
        const uint32_t z = f ^ canon;
        const uint32_t bad = (((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z) & 0x80808080u;  // byte != letter
        code |= ((d * 0x40100401u) >> 24) << (24 - 8 * q);
        valid |= ((((bad ^ 0x80808080u) >> 7) * 0x80402010u) >> 28) << (28 - 4 * q);
    }
}

// Id of the k-mer whose first base is tile byte idx. win64[m] holds the
// digits of chunks m and m+1 (32 bases, first base in the top bits) and
// val32[m] their validity bits, so any k-mer (k <= 15) starting in chunk m
// is one shift of win64[m] and one of val32[m].
__device__ __forceinline__ int32_t kmer_at(const uint64_t *win64, const uint32_t *val32, uint32_t idx, int32_t k) {
    const uint32_t w = idx >> 4, o = idx & 15;
    const uint32_t digits = (uint32_t)(win64[w] >> (64 - 2 * (o + (uint32_t)k))) & ((1u << (2 * k)) - 1);
    const uint32_t km = (1u << k) - 1;
    const bool ok = ((val32[w] >> (32 - o - (uint32_t)k)) & km) == km;
    return ok ? (int32_t)(5 + digits) : DNATOK_ID_UNK;
}

// A relative cell index, or -1 when it lies before the segment (single
// cells: CLS, SEP, short final frame).
__device__ __forceinline__ int32_t clamp_rel(int64_t v, int64_t hi) {
    return (int32_t)(v < -1 ? -1 : (v > hi ? hi : v));
}
// A bound of a relative cell range, clamped to the segment [0, hi].
__device__ __forceinline__ int32_t clamp_cells(int64_t v, int64_t hi) {
    return (int32_t)(v < 0 ? 0 : (v > hi ? hi : v));
}

// ---- row scan ------------------------------------------------------------------

struct RowScanArgs {
    const int64_t *offs;
    int32_t n;
    int64_t nbytes;
    int64_t *out_offs;
    int32_t k;
    int32_t kmer;
    int32_t cls;
    int32_t padded;
    int64_t W;
    int64_t base;
    int64_t nunits;
    dev::TileQueue q;
};

// Lengths of the up-to-kUnitRows rows starting at row0 (validated), their
// exclusive scan written to out_offs after `Prefix(total)` supplies the
// unit's starting value. Returns the unit's token total.
template <class Prefix>
__device__ __forceinline__ int64_t rowscan_unit(const RowScanArgs &a, int64_t row0, int64_t *s_tmp, uint32_t &err,
                                                Prefix prefix) {
    const int tid = threadIdx.x;
    const int64_t i0 = row0 + (int64_t)tid * kRowsPerThread;
    int64_t len[kRowsPerThread];
    int64_t mine = 0;
#pragma unroll
    for (int j = 0; j < kRowsPerThread; ++j) {
        const int64_t i = i0 + j;
        len[j] = 0;
        if (i < a.n) {
            int64_t o0 = a.offs[i], o1 = a.offs[i + 1];
            if (o0 < 0 || o1 < o0 || o1 > a.nbytes) err |= DNATOK_DERR_OFFSETS;
            o0 = o0 < 0 ? 0 : (o0 > a.nbytes ? a.nbytes : o0);
            o1 = o1 < o0 ? o0 : (o1 > a.nbytes ? a.nbytes : o1);
            len[j] = body_tokens(o1 - o0, a.k, a.kmer) + 2 * a.cls;
            if (a.padded && len[j] > a.W) err |= DNATOK_DERR_ROW_WIDTH;
        }
        mine += len[j];
    }
    int64_t total;
    const int64_t pre = dev::block_excl_scan<NT>(mine, s_tmp, &total);
    int64_t run = a.base + prefix(total) + pre;
#pragma unroll
    for (int j = 0; j < kRowsPerThread; ++j) {
        const int64_t i = i0 + j;
        if (i < a.n) a.out_offs[i] = run;
        run += len[j];
    }
    return total;
}

// Whole batch by one block, units in order (the fused PADDED case).
__device__ void rowscan_single_block(const RowScanArgs &a, int64_t *s_tmp, uint32_t *err_hdr) {
    uint32_t err = 0;
    int64_t run = 0;
    for (int64_t row0 = 0; row0 < a.n; row0 += kUnitRows) {
        rowscan_unit(a, row0, s_tmp, err, [&](int64_t total) {
            const int64_t b = run;
            run += total;
            return b;
        });
    }
    if (threadIdx.x == 0) a.out_offs[a.n] = a.base + run;
    if (err) dev::raise_error(err_hdr, err);
}

__global__ __launch_bounds__(NT) void k_rowscan(RowScanArgs a) {
    __shared__ int64_t s_tmp[NT / dev::kWave + 1];
    __shared__ int64_t s_unit, s_excl;
    const int tid = threadIdx.x;
    const uint32_t parity = dev::ld_relaxed32(a.q.hdr + 2);
    uint64_t *st = parity ? a.q.status1 : a.q.status0;
    uint64_t *st_other = parity ? a.q.status0 : a.q.status1;
    uint32_t err = 0;
    for (;;) {
        if (tid == 0) s_unit = (int64_t)atomicAdd(a.q.hdr + 0, 1u);
        __syncthreads();
        const int64_t u = s_unit;
        __syncthreads();
        if (u >= a.nunits) break;
        for (int64_t j = u + (int64_t)tid * a.nunits; j < a.q.clear_n; j += (int64_t)NT * a.nunits) st_other[j] = 0;
        // Unit prefix through the decoupled look-back over units (wave 0).
        const int64_t total = rowscan_unit(a, u * kUnitRows, s_tmp, err, [&](int64_t tot) {
            if (threadIdx.x < dev::kWave) {
                if (threadIdx.x == 0) dev::publish_aggregate(st, u, tot);
                const int64_t ex = dev::wave_lookback(st, u, tot);
                if (threadIdx.x == 0) s_excl = ex;
            }
            __syncthreads();
            return s_excl;
        });
        if (u == a.nunits - 1 && tid == 0) a.out_offs[a.n] = a.base + s_excl + total;
        __syncthreads();
    }
    if (err) dev::raise_error(a.q.hdr, err);
    if (tid == 0) dev::finish_block(a.q.hdr);
}

// ---- cell kernel -------------------------------------------------------------------

// One vocabulary's output of a cell launch (several k-mer vocabularies can
// share one pass over the input).
struct VocabOut {
    int32_t k;
    int32_t al;               // element misalignment of ids within 16 bytes
    int32_t *ids;
    int64_t cap;
    const int64_t *out_offs;  // PACKED: row starts (written by the row scan)
    int64_t *out_offs_w;      // the same array, written by a fused packed scan
    int8_t *mask;
    const int32_t *lut;
    int32_t pad_id, cls_id, sep_id;
    int64_t W;
    int64_t base;
};

struct CellArgs {
    const uint8_t *abase;  // input base aligned down to 16 bytes
    int64_t shift;         // d_bytes - abase
    int64_t nbytes;
    const int64_t *offs;
    int32_t n;
    int32_t nv;            // vocabularies written by this launch
    int32_t cls;
    int32_t padded;
    int32_t left;
    int64_t tileB;
    int64_t ntiles;
    int32_t fused_scan;  // the last block runs the row scans instead of tiles
    int32_t fused_packed;   // PACKED, <= kFusePackedRows rows: each block scans the row lengths into LDS
    int32_t prefix_off;     // byte offset of that scan in the dynamic LDS
    uint32_t *err_hdr;
    VocabOut vo[kMaxMultiVocabs];
    RowScanArgs scan[kMaxMultiVocabs];
};

// Per-row facts a tile needs for its owned cells (row chunk of up to NT rows).
struct SegInfo {
    int64_t dlo;       // destination element of the first owned cell
    int64_t gpre;      // first 4-element store group of this segment in the chunk's group list
    int64_t base_idx;  // tile-relative byte index of the body token at relative cell 0
    int32_t ncell;     // owned cells
    int32_t b0, b1;    // relative cells holding body tokens
    int32_t cc_cls, cc_sep, cc_tail;  // relative cells of CLS, SEP and a short final k-mer (-1 if none)
};

__device__ __forceinline__ uint4 load_chunk(const CellArgs &a, int64_t q0) {
    if (q0 >= a.shift && q0 + 16 <= a.shift + a.nbytes)
        return *reinterpret_cast<const uint4 *>(a.abase + q0);
    uint32_t w[4] = {0, 0, 0, 0};
    for (int b = 0; b < 16; ++b) {
        int64_t qb = q0 + b;
        if (qb >= a.shift && qb < a.shift + a.nbytes) w[b >> 2] |= (uint32_t)a.abase[qb] << (8 * (b & 3));
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Put the 16-byte chunks of tile t that this thread stages in flight:
// chunk u * NT + tid for u < U, plus (thread 0) the halo chunk U * NT that
// holds the first bytes of the next tile. Tiles whose chunks all lie inside
// the input take branch-free vector loads; only the first and last tile
// check bytes one by one.
template <int U>
__device__ __forceinline__ void fetch_tile(const CellArgs &a, int64_t t, uint4 (&v)[U], uint4 &halo) {
    const int tid = threadIdx.x;
    constexpr int64_t nchunks = (int64_t)U * NT + 1;
    const bool interior = (t * a.tileB >= a.shift) && (t * a.tileB + nchunks * 16 <= a.shift + a.nbytes);
    if (interior) {
        const u32x4 *src = reinterpret_cast<const u32x4 *>(a.abase + t * a.tileB);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const u32x4 x = __builtin_nontemporal_load(src + (int64_t)u * NT + tid);
            v[u] = make_uint4(x[0], x[1], x[2], x[3]);
        }
        if (tid == 0) {
            const u32x4 x = __builtin_nontemporal_load(src + (int64_t)U * NT);
            halo = make_uint4(x[0], x[1], x[2], x[3]);
        }
    } else {
        for (int u = 0; u < U; ++u) v[u] = load_chunk(a, t * a.tileB + 16 * ((int64_t)u * NT + tid));
        if (tid == 0) halo = load_chunk(a, t * a.tileB + 16 * (int64_t)U * NT);
    }
}

template <bool KMER, int U>
__global__ __launch_bounds__(NT) void k_cells(CellArgs a) {
    extern __shared__ __align__(16) uint8_t dyn[];
    __shared__ int32_t lut_s[256];
    __shared__ SegInfo seg[NT];
    __shared__ int64_t s_tmp[NT / dev::kWave + 1];
    __shared__ int64_t s_ia, s_ib;
    __shared__ uint32_t s_err;

    const int tid = threadIdx.x;
    if (a.fused_scan && blockIdx.x == gridDim.x - 1) {
        for (int vi = 0; vi < a.nv; ++vi) {
            rowscan_single_block(a.scan[vi], s_tmp, a.err_hdr);
            __syncthreads();
        }
        return;
    }
    const int64_t G = gridDim.x - (a.fused_scan ? 1 : 0);
    if (!KMER)
        for (int i = tid; i < 256; i += NT) lut_s[i] = a.vo[0].lut[i];
    if (tid == 0) s_err = 0;
    const int64_t B = a.tileB;  // == U * NT * 16
    constexpr int64_t nchunks = (int64_t)U * NT + 1;
    uint64_t *win64 = reinterpret_cast<uint64_t *>(dyn);                 // KMER: nchunks
    uint32_t *val32 = reinterpret_cast<uint32_t *>(win64 + nchunks);     // KMER: nchunks
    uint8_t *raw = dyn;
    const int64_t off_first = (a.n > 0) ? a.offs[0] : 0;
    const int64_t off_last = (a.n > 0) ? a.offs[a.n] : 0;
    uint32_t err = 0;
    int64_t *s_prefix = reinterpret_cast<int64_t *>(dyn + a.prefix_off);
    if (a.fused_packed) {
        // Small PACKED batch: every block forms the row starts itself (two
        // rows per thread) instead of waiting for a separate row-scan launch;
        // block 0 also publishes them as the output offsets.
        const VocabOut &o = a.vo[0];
        const int32_t kk = KMER ? o.k : 1;
        int64_t len2[2];
        int64_t mine = 0;
        uint32_t e2 = 0;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t i = 2 * (int64_t)tid + j;
            len2[j] = 0;
            if (i < a.n) {
                int64_t o0 = a.offs[i], o1 = a.offs[i + 1];
                if (o0 < 0 || o1 < o0 || o1 > a.nbytes) e2 |= DNATOK_DERR_OFFSETS;
                o0 = o0 < 0 ? 0 : (o0 > a.nbytes ? a.nbytes : o0);
                o1 = o1 < o0 ? o0 : (o1 > a.nbytes ? a.nbytes : o1);
                len2[j] = body_tokens(o1 - o0, kk, KMER) + 2 * a.cls;
            }
            mine += len2[j];
        }
        int64_t total;
        int64_t run = dev::block_excl_scan<NT>(mine, s_tmp, &total);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t i = 2 * (int64_t)tid + j;
            if (i < a.n) {
                s_prefix[i] = run;
                if (blockIdx.x == 0) o.out_offs_w[i] = o.base + run;
            }
            run += len2[j];
        }
        if (blockIdx.x == 0 && tid == 0) o.out_offs_w[a.n] = o.base + total;
        if (blockIdx.x == 0) err |= e2;
        __syncthreads();
    }

    auto load_row = [&](int64_t i, int32_t k) {
        Row r;
        int64_t o0 = a.offs[i], o1 = a.offs[i + 1];
        o0 = o0 < 0 ? 0 : (o0 > a.nbytes ? a.nbytes : o0);
        o1 = o1 < o0 ? o0 : (o1 > a.nbytes ? a.nbytes : o1);
        r.off = o0;
        r.end = o1;
        r.nb = body_tokens(o1 - o0, k, KMER);
        r.len = r.nb + 2 * a.cls;
        return r;
    };

    uint4 v[U];
    uint4 halo = make_uint4(0, 0, 0, 0);
    int64_t t = blockIdx.x;
    if (t < a.ntiles) fetch_tile<U>(a, t, v, halo);
    for (; t < a.ntiles; t += G) {
        const int64_t P0 = t * B - a.shift;
        const int64_t P1 = (t == a.ntiles - 1) ? INT64_MAX : P0 + B;

        // Stage this tile from registers into LDS, then put the next tile's
        // loads in flight while this one is written.
        auto stage = [&](int64_t m, uint4 x) {
            if (KMER) {
                // chunk m's digits are the high half of window m and the low
                // half of window m-1 (likewise its validity bits)
                uint32_t c, vb;
                classify16(x, c, vb);
                uint32_t *w32 = reinterpret_cast<uint32_t *>(win64);
                uint16_t *v16 = reinterpret_cast<uint16_t *>(val32);
                w32[2 * m + 1] = c;
                v16[2 * m + 1] = (uint16_t)(vb >> 16);
                if (m > 0) {
                    w32[2 * m - 2] = c;
                    v16[2 * m - 2] = (uint16_t)(vb >> 16);
                }
            } else {
                reinterpret_cast<uint4 *>(raw)[m] = x;
            }
        };
#pragma unroll
        for (int u = 0; u < U; ++u) stage((int64_t)u * NT + tid, v[u]);
        if (tid == 0) stage(nchunks - 1, halo);
        if (t + G < a.ntiles) fetch_tile<U>(a, t + G, v, halo);

        // Wave 0: rows with an anchor in [P0, P1) are [ia, ib). The first
        // probe window is centred on the row the byte position would fall in
        // if rows were equally long; a miss falls back to a 64-way search.
        if (tid < dev::kWave) {
            auto pa = [&](int64_t i) {
                const int64_t o0 = a.offs[i], o1 = a.offs[i + 1];
                return ((o1 > o0) ? o1 - 1 : o0) >= P0;
            };
            auto pb = [&](int64_t i) { return a.offs[i] >= P1; };
            const int64_t n = a.n;
            int64_t guess = 0;
            if (off_last > off_first && P0 > off_first)
                guess = (int64_t)((double)(P0 - off_first) / (double)(off_last - off_first) * (double)n);
            int64_t w0 = guess - dev::kWave / 2;
            if (w0 + dev::kWave > n) w0 = n - dev::kWave;
            if (w0 < 0) w0 = 0;
            const int64_t w1 = (w0 + dev::kWave < n) ? w0 + dev::kWave : n;  // probe [w0, w1)
            const int64_t q = w0 + tid;
            const bool live = q < w1;
            const uint64_t ba = __ballot(live ? pa(q) : true);
            int64_t ia;
            if (w0 > 0 && (ba & 1ull)) ia = dev::wave_lower_bound(0, w0, pa);  // answer left of the window
            else ia = ba ? w0 + __builtin_ctzll(ba) : w1;  // inside, or w1 == n
            if (ia == w1 && w1 < n) ia = dev::wave_lower_bound(w1, n, pa);  // right of the window
            int64_t ib = n;
            if (P1 != INT64_MAX) {
                // pb is monotone too and its answer is >= ia; reuse the window when it brackets it
                const uint64_t bb = __ballot(live && q >= ia ? pb(q) : (q >= ia));
                const int64_t lo = ia > w0 ? ia : w0;
                if (lo < w1 && ia >= w0 && bb) {
                    const int64_t cand = w0 + __builtin_ctzll(bb);
                    ib = (cand < w1) ? cand : dev::wave_lower_bound(w1, n, pb);
                } else {
                    ib = dev::wave_lower_bound(ia, n, pb);
                }
            }
            if (tid == 0) {
                s_ia = ia;
                s_ib = ib;
            }
        }
        __syncthreads();
        const int64_t ia = s_ia, ib = s_ib;

        // Write pass per vocabulary, one chunk of up to NT rows at a time.
        for (int vi = 0; vi < a.nv; ++vi) {
        const VocabOut &o = a.vo[vi];
        const int32_t k = KMER ? o.k : 1;
        const int64_t al = o.al;
        for (int64_t cb = ia; cb < ib; cb += NT) {
            const int64_t i = cb + tid;
            const int nrows = (int)((ib - cb) < NT ? (ib - cb) : NT);
            int64_t gcnt = 0;
            if (i < ib) {
                const Row r = load_row(i, k);
                int64_t clo = 0, chi = 0;
                if (!(a.padded && r.len > o.W)) {
                    clo = cells_before(r, P0, k, a.cls, a.padded, a.left, o.W);
                    chi = cells_before(r, P1, k, a.cls, a.padded, a.left, o.W);
                }
                const int64_t ncell = chi - clo;
                const int64_t lead = (a.padded && a.left) ? o.W - r.len : 0;
                const int64_t tt0 = clo - lead;  // token index of the first owned cell
                SegInfo sg;
                sg.ncell = (int32_t)ncell;
                sg.b0 = clamp_cells(a.cls - tt0, ncell);
                sg.b1 = clamp_cells(a.cls + r.nb - tt0, ncell);
                sg.cc_cls = a.cls ? clamp_rel(-tt0, ncell) : -1;
                sg.cc_sep = a.cls ? clamp_rel(r.len - 1 - tt0, ncell) : -1;
                sg.cc_tail = (KMER && r.nb > 0 && (r.end - r.off) % k) ? clamp_rel(a.cls + r.nb - 1 - tt0, ncell) : -1;
                sg.base_idx = (r.off - P0) + (tt0 - a.cls) * k;
                sg.dlo = a.padded ? i * o.W + clo : (a.fused_packed ? s_prefix[i] : o.out_offs[i] - o.base) + clo;
                sg.gpre = 0;
                seg[tid] = sg;
                if (ncell > 0) gcnt = ((sg.dlo + al + ncell - 1) >> 2) - ((sg.dlo + al) >> 2) + 1;
            }
            int64_t G4;
            const int64_t gpre = dev::block_excl_scan<NT>(gcnt, s_tmp, &G4);
            if (i < ib) seg[tid].gpre = gpre;
            __syncthreads();

            // Groups walk segments in order: cache the current segment's facts
            // in registers and reload them only when a group crosses into
            // another segment.
            int s = -1;
            int64_t seg_lo = 0, seg_hi = -1;  // groups [seg_lo, seg_hi) belong to segment s
            SegInfo sg{};
            int64_t gb = 0;      // aligned group index of the segment's first group, minus gpre
            int32_t ccb = 0;     // relative cell of the first element of group qi = ccb + 4 * (qi - seg_lo)
            for (int64_t qi = tid; qi < G4; qi += NT) {
                if (qi < seg_lo || qi >= seg_hi) {
                    int lo = 0, hi = nrows - 1;
                    while (lo < hi) {  // last segment with gpre <= qi
                        int mid = (lo + hi + 1) >> 1;
                        if (seg[mid].gpre <= qi) lo = mid;
                        else hi = mid - 1;
                    }
                    s = lo;
                    sg = seg[s];
                    seg_lo = sg.gpre;
                    seg_hi = (s + 1 < nrows) ? seg[s + 1].gpre : G4;
                    gb = ((sg.dlo + al) >> 2) - sg.gpre;
                    ccb = (int32_t)((((sg.dlo + al) >> 2) * 4 - al) - sg.dlo);
                }
                const int64_t eb = (gb + qi) * 4 - al;
                const int32_t cc0 = ccb + 4 * (int32_t)(qi - seg_lo);
                int32_t *dst = o.ids + eb;
                // Fast path: four body tokens, none of them a short final frame.
                const bool fast = cc0 >= sg.b0 && cc0 + 3 < sg.b1 && (uint32_t)(sg.cc_tail - cc0) > 3u &&
                                  (a.padded || (eb >= 0 && eb + 3 < o.cap));
                if (fast) {
                    const uint32_t idx0 = (uint32_t)sg.base_idx + (uint32_t)cc0 * (uint32_t)k;
                    int32_t vv[4];
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const uint32_t idx = idx0 + (uint32_t)(rr * k);
                        if (KMER) vv[rr] = kmer_at(win64, val32, idx, k);
                        else vv[rr] = lut_s[raw[idx]];
                    }
                    i32x4 x = {vv[0], vv[1], vv[2], vv[3]};
                    __builtin_nontemporal_store(x, reinterpret_cast<i32x4 *>(dst));
                    if (a.padded) {
                        int8_t *md = o.mask + eb;
                        if ((reinterpret_cast<uintptr_t>(md) & 3) == 0)
                            __builtin_nontemporal_store(0x01010101u, reinterpret_cast<uint32_t *>(md));
                        else
                            for (int rr = 0; rr < 4; ++rr) md[rr] = 1;
                    }
                    continue;
                }
                int32_t vv[4];
                uint32_t mk = 0;
                bool in[4];
                bool all_in = true;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int32_t cc = cc0 + rr;
                    in[rr] = (cc >= 0 && cc < sg.ncell);
                    if (in[rr] && !a.padded && (eb + rr < 0 || eb + rr >= o.cap)) {
                        in[rr] = false;
                        err |= DNATOK_DERR_CAPACITY;
                    }
                    all_in = all_in && in[rr];
                    int32_t val = o.pad_id;
                    uint32_t m = 0;
                    if (in[rr]) {
                        if (cc >= sg.b0 && cc < sg.b1) {
                            m = 1;
                            const uint32_t idx = (uint32_t)sg.base_idx + (uint32_t)cc * (uint32_t)k;
                            if (KMER) val = (cc == sg.cc_tail) ? DNATOK_ID_UNK : kmer_at(win64, val32, idx, k);
                            else val = lut_s[raw[idx]];
                        } else if (cc == sg.cc_cls) {
                            val = o.cls_id;
                            m = 1;
                        } else if (cc == sg.cc_sep) {
                            val = o.sep_id;
                            m = 1;
                        }
                    }
                    vv[rr] = val;
                    mk |= m << (8 * rr);
                }
                if (all_in) {
                    *reinterpret_cast<int4 *>(dst) = make_int4(vv[0], vv[1], vv[2], vv[3]);
                    if (a.padded) {
                        int8_t *md = o.mask + eb;
                        if ((reinterpret_cast<uintptr_t>(md) & 3) == 0) {
                            *reinterpret_cast<uint32_t *>(md) = mk;
                        } else {
#pragma unroll
                            for (int rr = 0; rr < 4; ++rr) md[rr] = (int8_t)((mk >> (8 * rr)) & 1);
                        }
                    }
                } else {
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        if (!in[rr]) continue;
                        dst[rr] = vv[rr];
                        if (a.padded) o.mask[eb + rr] = (int8_t)((mk >> (8 * rr)) & 1);
                    }
                }
            }
            __syncthreads();
        }
        }
    }
    if (err) atomicOr(&s_err, err);
    __syncthreads();
    if (tid == 0 && s_err) dev::raise_error(a.err_hdr, s_err);
}

template <bool KMER>
int launch_cells(const CellArgs &a, int U, int64_t grid, size_t dyn, hipStream_t stream) {
    switch (U) {
    case 1: hipLaunchKernelGGL((k_cells<KMER, 1>), dim3((unsigned)grid), dim3(NT), dyn, stream, a); break;
    case 2: hipLaunchKernelGGL((k_cells<KMER, 2>), dim3((unsigned)grid), dim3(NT), dyn, stream, a); break;
    case 4: hipLaunchKernelGGL((k_cells<KMER, 4>), dim3((unsigned)grid), dim3(NT), dyn, stream, a); break;
    case 8: hipLaunchKernelGGL((k_cells<KMER, 8>), dim3((unsigned)grid), dim3(NT), dyn, stream, a); break;
    case 16: hipLaunchKernelGGL((k_cells<KMER, 16>), dim3((unsigned)grid), dim3(NT), dyn, stream, a); break;
    default: return set_error(DNATOK_EINVAL, "unsupported staging depth %d", U);
    }
    DNATOK_HIP(hipGetLastError());
    return DNATOK_OK;
}

template <bool KMER>
int blocks_per_cu(int U, size_t dyn, int *out) {
    *out = 1;
    switch (U) {
    case 1: DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_cells<KMER, 1>, NT, dyn)); break;
    case 2: DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_cells<KMER, 2>, NT, dyn)); break;
    case 4: DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_cells<KMER, 4>, NT, dyn)); break;
    case 8: DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_cells<KMER, 8>, NT, dyn)); break;
    case 16: DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_cells<KMER, 16>, NT, dyn)); break;
    default: break;
    }
    return DNATOK_OK;
}

}  // namespace

int launch_rowscan(const int64_t *d_offsets, int32_t n, int64_t nbytes, int64_t *d_out, int32_t divisor, int32_t cls,
                   hipStream_t stream) {
    RowScanArgs s;
    s.offs = d_offsets;
    s.n = n;
    s.nbytes = nbytes;
    s.out_offs = d_out;
    s.k = divisor;
    s.kmer = 1;
    s.cls = cls;
    s.padded = 0;
    s.W = 0;
    s.base = 0;
    s.nunits = ((int64_t)n + kUnitRows - 1) / kUnitRows;
    if (s.nunits < 1) s.nunits = 1;
    Workspace *ws = nullptr;
    int rc = get_workspace(stream, s.nunits, &ws);
    if (rc) return rc;
    s.q.hdr = ws->d_hdr;
    s.q.status0 = ws->d_status;
    s.q.status1 = ws->d_status + ws->cap;
    if (s.nunits > ws->high_water) ws->high_water = s.nunits;
    s.q.clear_n = ws->high_water;
    int per_cu = 0;
    DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rowscan, NT, 0));
    int64_t g = (int64_t)device_cu_count() * (per_cu > 0 ? per_cu : 1);
    if (g > s.nunits) g = s.nunits;
    hipLaunchKernelGGL(k_rowscan, dim3((unsigned)g), dim3(NT), 0, stream, s);
    DNATOK_HIP(hipGetLastError());
    return DNATOK_OK;
}

EncodeTuning encode_tuning(const dnatok_vocab *v) {
    const bool kmer = (v->kind == DNATOK_KMER);
    EncodeTuning t;
    const int32_t tile = v->tune_tile.load(std::memory_order_relaxed);
    t.tile_bytes = tile > 0 ? tile : (kmer ? 32768 : 16384);
    t.blocks_per_cu = v->tune_blocks.load(std::memory_order_relaxed);
    return t;
}

int launch_encode_multi(const dnatok_vocab *const *vs, int nv, const uint8_t *d_bytes, int64_t nbytes,
                        const int64_t *d_offsets, int32_t n, int32_t *const *d_ids, const int64_t *caps,
                        int64_t *const *d_out_offsets, int8_t *const *d_masks, const dnatok_encode_opts *os,
                        hipStream_t stream) {
    if (nv < 1 || nv > kMaxMultiVocabs) return set_error(DNATOK_EINVAL, "1 to %d vocabularies", kMaxMultiVocabs);
    const dnatok_vocab *v = vs[0];
    const dnatok_encode_opts &o = os[0];
    const bool kmer = (v->kind == DNATOK_KMER);
    const EncodeTuning tune = encode_tuning(v);
    int U = 1;  // staging loads per thread: tiles are U * NT * 16 bytes
    while (U < 16 && (int64_t)U * NT * 16 < tune.tile_bytes) U <<= 1;
    const int64_t B = (int64_t)U * NT * 16;
    const int64_t nchunks = B / 16 + 1;

    CellArgs a;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(d_bytes);
    a.shift = (int64_t)(addr & 15);
    a.abase = d_bytes ? d_bytes - a.shift : nullptr;
    a.nbytes = nbytes;
    a.offs = d_offsets;
    a.n = n;
    a.nv = nv;
    a.cls = o.add_cls_sep ? 1 : 0;
    a.padded = (o.layout == DNATOK_PADDED) ? 1 : 0;
    a.left = (o.pad_side == DNATOK_PAD_LEFT) ? 1 : 0;
    a.tileB = B;
    // the last tile also owns the end position (anchors of trailing empty rows)
    a.ntiles = (nbytes + a.shift + B - 1) / B;
    if (a.ntiles < 1) a.ntiles = 1;
    const int64_t nunits = std::max<int64_t>(1, ((int64_t)n + kUnitRows - 1) / kUnitRows);

    Workspace *ws = nullptr;
    int rc = get_workspace(stream, nunits, &ws);
    if (rc) return rc;
    a.err_hdr = ws->d_hdr;
    a.fused_scan = (a.padded && n <= kFuseMaxRows) ? 1 : 0;
    a.fused_packed = (!a.padded && nv == 1 && n <= kFusePackedRows) ? 1 : 0;
    for (int vi = 0; vi < nv; ++vi) {
        const dnatok_vocab *w = vs[vi];
        VocabOut &out = a.vo[vi];
        out.k = kmer ? w->k : 1;
        out.al = (int32_t)((reinterpret_cast<uintptr_t>(d_ids[vi]) >> 2) & 3);
        out.ids = d_ids[vi];
        out.cap = caps[vi];
        out.out_offs = d_out_offsets[vi];
        out.out_offs_w = d_out_offsets[vi];
        out.mask = d_masks[vi];
        out.lut = w->d_lut;
        out.pad_id = w->pad_id;
        out.cls_id = w->cls_id;
        out.sep_id = w->sep_id;
        out.W = a.padded ? os[vi].pad_to : 0;
        out.base = os[vi].offset_base;

        RowScanArgs &sc = a.scan[vi];
        sc.offs = d_offsets;
        sc.n = n;
        sc.nbytes = nbytes;
        sc.out_offs = d_out_offsets[vi];
        sc.k = out.k;
        sc.kmer = kmer ? 1 : 0;
        sc.cls = a.cls;
        sc.padded = a.padded;
        sc.W = out.W;
        sc.base = out.base;
        sc.nunits = nunits;
        if (!a.fused_scan && !a.fused_packed) {
            sc.q.hdr = ws->d_hdr;
            sc.q.status0 = ws->d_status;
            sc.q.status1 = ws->d_status + ws->cap;
            if (sc.nunits > ws->high_water) ws->high_water = sc.nunits;
            sc.q.clear_n = ws->high_water;
            int per_cu = 0;
            DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rowscan, NT, 0));
            int64_t g = (int64_t)device_cu_count() * (per_cu > 0 ? per_cu : 1);
            if (g > sc.nunits) g = sc.nunits;
            hipLaunchKernelGGL(k_rowscan, dim3((unsigned)g), dim3(NT), 0, stream, sc);
            DNATOK_HIP(hipGetLastError());
        }
    }

    const size_t dyn_tile = ((kmer ? (size_t)nchunks * 12 : (size_t)nchunks * 16) + 15) / 16 * 16;
    a.prefix_off = (int32_t)dyn_tile;
    const size_t dyn = dyn_tile + (a.fused_packed ? 8 * (size_t)(n + 1) : 0);
    int per_cu = 0;
    rc = kmer ? blocks_per_cu<true>(U, dyn, &per_cu) : blocks_per_cu<false>(U, dyn, &per_cu);
    if (rc) return rc;
    if (per_cu < 1) per_cu = 1;
    if (tune.blocks_per_cu > 0 && tune.blocks_per_cu < per_cu) per_cu = tune.blocks_per_cu;
    // As many blocks as fit, then evened out so every block walks the same
    // number of tiles (no straggler round).
    const int64_t gmax = (int64_t)device_cu_count() * per_cu;
    const int64_t per_block = (a.ntiles + gmax - 1) / gmax;
    int64_t grid = (a.ntiles + per_block - 1) / per_block;
    if (a.fused_scan) grid += 1;
    return kmer ? launch_cells<true>(a, U, grid, dyn, stream) : launch_cells<false>(a, U, grid, dyn, stream);
}

int launch_encode(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                  int32_t n, int32_t *d_ids, int64_t cap, int64_t *d_out_offsets, int8_t *d_mask,
                  const dnatok_encode_opts &o, hipStream_t stream) {
    return launch_encode_multi(&v, 1, d_bytes, nbytes, d_offsets, n, &d_ids, &cap, &d_out_offsets, &d_mask, &o,
                               stream);
}

}  // namespace dnatok
