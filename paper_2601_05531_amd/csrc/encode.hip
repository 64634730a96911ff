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
//    (PADDED), so tiles never wait on each other: tile walkers take an
//    evened-out static share of the tiles, each XCD a contiguous range,
//    with no atomics at all (one ticket counter for the whole device is far
//    slower than any imbalance it would fix on this chip).
//  * Each tile is staged into LDS once with coalesced 16-byte loads, issued
//    together with the row-search probe so one wait covers both; walkers
//    with several tiles issue the next tile's loads before writing the
//    current one. k-mer tiles are classified on the way in: 2-bit base
//    digits packed most-significant-first (16 bases per word) plus one
//    validity bit per base. Single-base tiles keep raw bytes, with the
//    256-entry table in LDS.
//  * One pass over the rows of a chunk gives every (vocabulary, row) segment
//    of the tile; one block scan splits their aligned 16-byte store groups
//    into interior groups (four body tokens) and edge groups (specials,
//    pads, tails, ragged ends). Each wave writes a contiguous share of the
//    interior groups with the segment's facts uniform across it: four
//    k-mer ids from one 32-base window read, one 16-byte id store and one
//    4-byte mask word. Edge groups go cell by cell.
//  * PADDED layout with a modest row count folds the row scans into the
//    cell launch: its last nv blocks scan one vocabulary each.
#include "common.hpp"
#include "device.hpp"
#include "rowscan.hpp"

namespace dnatok {

namespace {

constexpr int NT = 256;
static_assert(NT == kScanNT, "the row scan runs with the cell kernel's block size");
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
__device__ __forceinline__ int64_t tokens_before(const Row &r, int64_t X, int32_t k, uint32_t kinv, int32_t cls) {
    int64_t c = 0;
    if (X > r.off) {
        // body anchors off + j*k < X  <=>  j < ceil((X - off) / k)
        c += (X >= r.end) ? r.nb : div_k(X - r.off + k - 1, k, kinv);
        if (cls) c += 1;  // CLS anchored at off
    }
    if (cls) {
        int64_t sep_anchor = (r.end > r.off) ? r.end - 1 : r.off;
        if (sep_anchor < X) c += 1;
    }
    return c;
}

// Cells (tokens plus pads) of the row whose anchor is < X.
__device__ __forceinline__ int64_t cells_before(const Row &r, int64_t X, int32_t k, uint32_t kinv, int32_t cls,
                                                int32_t padded, int32_t left, int64_t W) {
    int64_t c = tokens_before(r, X, k, kinv, cls);
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

// Per-vocabulary constants of kmer4_at: the shift that brings k-mer r of a
// 32-base window to the bottom, the validity bits it needs, the digit mask.
struct Kmer4 {
    uint32_t sh[4];
    uint32_t vm[4];
    uint32_t dm;
};

__device__ __forceinline__ Kmer4 kmer4_consts(int32_t k) {
    Kmer4 c;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        c.sh[r] = 64u - 2u * (uint32_t)(k * (r + 1));
        c.vm[r] = ((1u << k) - 1u) << (32 - k * (r + 1));
    }
    c.dm = (1u << (2 * k)) - 1u;
    return c;
}

// Ids of the four consecutive k-mers (k <= 8) starting at tile byte idx0.
// Their 4k bases lie within the 32 bases from idx0 on: window w = idx0 / 16
// shifted left by o = idx0 % 16 bases, with the first o bases of chunk w + 2
// (the low half of window w + 1) shifted in below; validity bits likewise.
__device__ __forceinline__ i32x4 kmer4_at(const uint64_t *win64, const uint32_t *val32, uint32_t idx0,
                                          const Kmer4 &c) {
    const uint32_t w = idx0 >> 4, o = idx0 & 15;
    const uint64_t w0 = win64[w], w1 = win64[w + 1];
    const uint32_t v0 = val32[w], v1 = val32[w + 1];
    const uint64_t X = (w0 << (2 * o)) | (((uint64_t)(uint32_t)w1 << (2 * o)) >> 32);
    const uint32_t nV = ~(uint32_t)((((uint64_t)v0 << 32) | (uint64_t)(v1 << 16)) << o >> 32);
    i32x4 r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int32_t id = 5 + (int32_t)((uint32_t)(X >> c.sh[q]) & c.dm);
        r[q] = (nV & c.vm[q]) == 0 ? id : DNATOK_ID_UNK;
    }
    return r;
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
                const int64_t ex = dev::wave_lookback(st, u, tot, a.q.hdr);
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
    uint32_t kinv;            // floor((2^32 - 1) / k)
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
    int32_t lut_off;        // byte offset of the 256-entry table in the dynamic LDS (SINGLE, LUT256)
    // Ticketed tiles (nticket > 0): blocks [0, lead) run the fused row scans
    // (the first nv of them) or nothing; tile block b = blockIdx - lead takes
    // tile xcd_tile(b, nstat) when b < nstat, else the next ticket's tile
    // nstat + ticket, or nothing once the tickets pass the last tile.
    int32_t lead;
    int64_t nstat;
    int64_t nticket;        // blocks that take a ticket (the last one resets the counter)
    uint32_t *ticket;
    uint32_t *err_hdr;
    VocabOut vo[kMaxMultiVocabs];
    RowScanArgs scan[kMaxMultiVocabs];
};

// Per-row facts a tile needs for its owned cells (row chunk of up to NT rows).
// Per-vocabulary facts the segment pass reads with a per-thread vocabulary
// index (kept in LDS: kernel arguments are read with uniform indices only).
struct VocabLds {
    int32_t k;
    uint32_t kinv;
    int32_t al;
    int32_t pad_;
    int64_t W;
    int64_t base;
    int64_t cap;
    const int64_t *out_offs;
};

struct SegInfo {
    int64_t dlo;        // destination element of the first owned cell
    int64_t epre;       // first edge group of this segment in the chunk's edge list
    uint32_t base_idx;  // tile-relative byte index (mod 2^32) of the body token at relative cell 0
    int32_t ncell;      // owned cells
    int32_t b0, b1;     // relative cells holding body tokens
    int32_t cc_cls, cc_sep, cc_tail;  // relative cells of CLS, SEP and a short final k-mer (-1 if none)
    int32_t ipre;       // first interior group of this segment in the chunk's interior list
};

// The aligned 4-element store groups of a segment whose first owned cell
// goes to element dlo (ids are 16-byte aligned at element -al): groups
// [gfirst, glast] touch it; [gA, gB) hold four body tokens, none of them the
// short final frame, and (PACKED) lie inside the capacity. The rest are its
// edge groups: [gfirst, gA) and [gB, glast].
struct SegGroups {
    int64_t gfirst, glast, gA, gB;
};

__device__ __forceinline__ SegGroups seg_groups(int64_t dlo, int64_t al, int32_t ncell, int32_t b0, int32_t b1,
                                                int32_t cc_tail, bool padded, int64_t cap) {
    SegGroups g;
    if (ncell <= 0) {
        g.gfirst = 0;
        g.glast = -1;
        g.gA = 0;
        g.gB = 0;
        return g;
    }
    g.gfirst = (dlo + al) >> 2;
    g.glast = (dlo + al + ncell - 1) >> 2;
    const int32_t fe = (cc_tail >= b0 && cc_tail < b1) ? cc_tail : b1;  // end of the full frames
    int64_t gA = (dlo + al + b0 + 3) >> 2;
    int64_t gB = (dlo + al + fe) >> 2;
    if (!padded) {
        const int64_t lo = (al + 3) >> 2, hi = (cap + al) >> 2;  // element 4g - al in [0, cap - 3]
        gA = gA > lo ? gA : lo;
        gB = gB < hi ? gB : hi;
    }
    if (gB < gA) gB = gA;
    g.gA = gA;
    g.gB = gB;
    return g;
}

__device__ __forceinline__ int32_t rfl(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t rfl64(int64_t v) {
    return (int64_t)(((uint64_t)(uint32_t)rfl((int32_t)(v >> 32)) << 32) | (uint32_t)rfl((int32_t)v));
}

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

// Workgroups are dispatched to the 8 XCDs in turn, so walk order L (tile
// walker bid takes L = bid, bid + G, ...) runs on XCD L % 8. Give each XCD a
// contiguous share of the tiles: neighbouring tiles, which share cache lines
// at their edges, then go through the same L2. A bijection on [0, ntiles).
__device__ __forceinline__ int64_t xcd_tile(int64_t L, int64_t ntiles) {
    const int64_t x = L & 7, j = L >> 3, q = ntiles >> 3, r = ntiles & 7;
    return x * q + (x < r ? x : r) + j;
}

// Whether every chunk of tile t, halo included, lies inside the input.
template <int U>
__device__ __forceinline__ bool tile_interior(const CellArgs &a, int64_t t) {
    constexpr int64_t nchunks = (int64_t)U * NT + 1;
    return (t * a.tileB >= a.shift) && (t * a.tileB + nchunks * 16 <= a.shift + a.nbytes);
}

// Put the 16-byte chunks of interior tile t that this thread stages in
// flight: chunk u * NT + tid for u < U, and the halo chunk U * NT holding the
// first bytes of the next tile (every thread loads it, one transaction per
// wave, so no value depends on the thread and nothing has to be merged).
template <int U>
__device__ __forceinline__ void fetch_tile(const CellArgs &a, int64_t t, uint4 (&v)[U], uint4 &halo, int tid) {
    const u32x4 *src = reinterpret_cast<const u32x4 *>(a.abase + t * a.tileB);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const u32x4 x = __builtin_nontemporal_load(src + (int64_t)u * NT + tid);
        v[u] = make_uint4(x[0], x[1], x[2], x[3]);
    }
    const u32x4 x = __builtin_nontemporal_load(src + (int64_t)U * NT);
    halo = make_uint4(x[0], x[1], x[2], x[3]);
}

// PF: blocks walk several tiles and the next tile's loads are issued while
// the current one is written (its registers stay live through the writes).
template <bool KMER, int U, bool PF>
__global__ __launch_bounds__(NT) void k_cells(CellArgs a) {
    extern __shared__ __align__(16) uint8_t dyn[];
    __shared__ SegInfo seg[NT];
    __shared__ VocabLds vtab[kMaxMultiVocabs];
    __shared__ int64_t s_vg[kMaxMultiVocabs + 1];
    __shared__ int64_t s_po[dev::kWave + 1];  // offs[s_w0 ..] as probed by the row search
    __shared__ int64_t s_w0, s_w1;
    __shared__ int32_t s_ipre[NT];  // first interior group of each (vocabulary, row) pair, in pair order
    __shared__ int64_t s_itot;
    __shared__ int64_t s_tmp[NT / dev::kWave + 1];
    __shared__ int64_t s_ia, s_ib;
    __shared__ uint32_t s_err;
    __shared__ uint32_t s_tk;

    const int tid = threadIdx.x;
    const int nscan = a.fused_scan ? a.nv : 0;
    int64_t bid, G;       // tile block index and the walkers' stride
    int64_t t_fixed = -1;  // ticketed launch: this block's one tile
    if (a.nticket > 0) {
        // Fused row scans first: every later block is a tile block, so they
        // never wait behind the tiles for a slot.
        if ((int64_t)blockIdx.x < a.lead) {
            if ((int)blockIdx.x < nscan) rowscan_single_block(a.scan[blockIdx.x], s_tmp, a.err_hdr);
            return;
        }
        bid = (int64_t)blockIdx.x - a.lead;
        if (bid < a.nstat) {
            t_fixed = xcd_tile(bid, a.nstat);
        } else {
            // Blocks that start late (a slot freed up) take the next tile in
            // line. Every ticket block takes exactly one ticket, so the one
            // that draws the last ticket can reset the counter for the next
            // launch: no block of this launch reads it again.
            if (tid == 0) {
                const uint32_t tk = atomicAdd(a.ticket, 1u);
                if ((int64_t)tk == a.nticket - 1) dev::st_relaxed32(a.ticket, 0u);
                s_tk = tk;
            }
            __syncthreads();
            const int64_t tk = s_tk;
            if (a.nstat + tk >= a.ntiles) return;  // an extra block with no tile left
            t_fixed = a.nstat + tk;
        }
        G = a.ntiles;  // one pass of the tile loop
    } else {
        // Fused PADDED row scans: the last nv blocks, one vocabulary each.
        // They start as the first tile walkers retire, so no walker waits
        // for a slot.
        G = (int64_t)gridDim.x - nscan;  // tile walkers
        if ((int64_t)blockIdx.x >= G) {
            rowscan_single_block(a.scan[blockIdx.x - G], s_tmp, a.err_hdr);
            return;
        }
        bid = blockIdx.x;
    }
    int32_t *lut_s = reinterpret_cast<int32_t *>(dyn + a.lut_off);
    if (!KMER)
        for (int i = tid; i < 256; i += NT) lut_s[i] = a.vo[0].lut[i];
    if (tid == 0) s_err = 0;
    for (int vi = 0; vi < a.nv; ++vi)
        if (tid == vi) {
            VocabLds e;
            e.k = a.vo[vi].k;
            e.kinv = a.vo[vi].kinv;
            e.al = a.vo[vi].al;
            e.pad_ = 0;
            e.W = a.vo[vi].W;
            e.base = a.vo[vi].base;
            e.cap = a.vo[vi].cap;
            e.out_offs = a.vo[vi].out_offs;
            vtab[vi] = e;
        }
    // rows per chunk: NT / nv rounded down to a power of two
    int R = NT;
    while (R * a.nv > NT) R >>= 1;
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
                if (bid == 0) o.out_offs_w[i] = o.base + run;
            }
            run += len2[j];
        }
        if (bid == 0 && tid == 0) o.out_offs_w[a.n] = o.base + total;
        if (bid == 0) err |= e2;
        __syncthreads();
    }

    auto make_row = [&](int64_t o0, int64_t o1, int32_t k, uint32_t kinv) {
        Row r;
        r.off = o0;
        r.end = o1;
        r.nb = KMER ? div_k(o1 - o0 + k - 1, k, kinv) : o1 - o0;
        r.len = r.nb + 2 * a.cls;
        return r;
    };

    uint4 v[U];
    uint4 halo = make_uint4(0, 0, 0, 0);
    // Row-search probe of the tile starting at byte P0: 64 rows around the
    // row that byte would fall in if rows were equally long, [w0, w1), and
    // (wave 0) the offsets bounding them, indices clamped to the batch.
    auto probe_window = [&](int64_t P0, int64_t &w0, int64_t &w1) {
        const int64_t n = a.n;
        int64_t guess = 0;
        if (off_last > off_first && P0 > off_first)
            guess = (int64_t)((double)(P0 - off_first) / (double)(off_last - off_first) * (double)n);
        w0 = guess - dev::kWave / 2;
        if (w0 + dev::kWave > n) w0 = n - dev::kWave;
        if (w0 < 0) w0 = 0;
        w1 = (w0 + dev::kWave < n) ? w0 + dev::kWave : n;
    };
    int64_t po0 = 0, po1 = 0;  // wave 0: offs[w0 + lane], offs[w0 + lane + 1] of the next probe
    auto probe_load = [&](int64_t P0) {
        if (tid < dev::kWave) {
            int64_t w0, w1;
            probe_window(P0, w0, w1);
            const int64_t q = w0 + tid;
            po0 = a.offs[q < a.n ? q : a.n];
            po1 = a.offs[q + 1 < a.n ? q + 1 : a.n];
        }
    };
    // v and halo hold tile t's chunks when pf is set; first and last tiles
    // (not interior) are read byte by byte when staged. With PF the next
    // tile's probe is put in flight with its bytes (probed).
    bool pf = false, probed = false;
    if (PF && t_fixed < 0 && bid < a.ntiles) {
        const int64_t t0 = xcd_tile(bid, a.ntiles);
        probe_load(t0 * B - a.shift);
        probed = true;
        pf = tile_interior<U>(a, t0);
        if (pf) fetch_tile<U>(a, t0, v, halo, tid);
    }
    for (int64_t L = (t_fixed >= 0 ? 0 : bid); L < a.ntiles; L += G) {
        const int64_t t = (t_fixed >= 0) ? t_fixed : xcd_tile(L, a.ntiles);
        // The staging addresses are recomputed per tile from a copy of the
        // thread index the compiler cannot see through: hoisted out of the
        // loop they would hold some 5 registers per chunk through the writes.
        int stid = tid;
        asm volatile("" : "+v"(stid));
        const int64_t P0 = t * B - a.shift;
        const int64_t P1 = (t == a.ntiles - 1) ? INT64_MAX : P0 + B;

        // Wave 0 puts the row search's probe in flight before the tile's own
        // loads (unless it went out with the prefetch), so one wait covers
        // both.
        int64_t w0 = 0, w1 = 0;
        probe_window(P0, w0, w1);
        if (!probed) probe_load(P0);
        probed = false;
        if (!PF) {
            pf = tile_interior<U>(a, t);
            if (pf) fetch_tile<U>(a, t, v, halo, stid);
        }

        // Stage this tile into LDS (from the registers its prefetch filled).
        auto stage = [&](int64_t m, uint4 x) {
            if (KMER) {
                // chunk m's digits are the high half of window m and the low
                // half of window m-1 (likewise its validity bits)
                uint32_t c, vb;
                dev::classify16(x, c, vb);
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
        if (pf) {
            // one chunk at a time: interleaving the classification of all U
            // chunks buys nothing and costs registers through the whole kernel
#pragma unroll
            for (int u = 0; u < U; ++u) {
                stage((int64_t)u * NT + stid, v[u]);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (stid == 0) stage(nchunks - 1, halo);
        } else {
            for (int u = 0; u < U; ++u)
                stage((int64_t)u * NT + stid, load_chunk(a, t * B + 16 * ((int64_t)u * NT + stid)));
            if (stid == 0) stage(nchunks - 1, load_chunk(a, t * B + 16 * (int64_t)U * NT));
        }

        // Wave 0: rows with an anchor in [P0, P1) are [ia, ib), from the
        // probed window when it brackets them, else by a 64-way search.
        if (tid < dev::kWave) {
            auto pa = [&](int64_t i) {
                const int64_t o0 = a.offs[i], o1 = a.offs[i + 1];
                return ((o1 > o0) ? o1 - 1 : o0) >= P0;
            };
            auto pb = [&](int64_t i) { return a.offs[i] >= P1; };
            const int64_t n = a.n;
            const int64_t q = w0 + tid;
            const bool live = q < w1;
            const uint64_t ba = __ballot(live ? (((po1 > po0) ? po1 - 1 : po0) >= P0) : true);
            int64_t ia;
            if (w0 > 0 && (ba & 1ull)) ia = dev::wave_lower_bound(0, w0, pa);  // answer left of the window
            else ia = ba ? w0 + __builtin_ctzll(ba) : w1;  // inside, or w1 == n
            if (ia == w1 && w1 < n) ia = dev::wave_lower_bound(w1, n, pa);  // right of the window
            int64_t ib = n;
            if (P1 != INT64_MAX) {
                // pb is monotone too and its answer is >= ia; reuse the window when it brackets it
                const uint64_t bb = __ballot(live && q >= ia ? (po0 >= P1) : (q >= ia));
                const int64_t lo = ia > w0 ? ia : w0;
                if (lo < w1 && ia >= w0 && bb) {
                    const int64_t cand = w0 + __builtin_ctzll(bb);
                    ib = (cand < w1) ? cand : dev::wave_lower_bound(w1, n, pb);
                } else {
                    ib = dev::wave_lower_bound(ia, n, pb);
                }
            }
            s_po[tid] = po0;
            if (tid == dev::kWave - 1) s_po[dev::kWave] = po1;
            if (tid == 0) {
                s_ia = ia;
                s_ib = ib;
                s_w0 = w0;
                s_w1 = w1;
            }
        }
        __syncthreads();
        const int64_t ia = s_ia, ib = s_ib;

        // Rows are taken in chunks of R rows, R = NT / nv rounded down to a
        // power of two, so every (vocabulary, row) pair of a chunk has a
        // thread: one segment pass and one block scan serve all vocabularies.
        // A chunk's byte offsets are read once, before any of its stores: a
        // vector load waits for all of the wave's earlier stores as well, so
        // a load between write passes would drain the write stream. The next
        // tile's loads go out after the first chunk's offsets and overlap this
        // tile's writes.
        const int pv = tid / R, pr = tid % R;  // this thread's (vocabulary, row-in-chunk) pair
        int64_t ro0 = 0, ro1 = 0;  // clamped byte range of row cb + pr
        const int64_t pw0 = s_w0, pw1 = s_w1;
        auto load_offs = [&](int64_t cb) {
            const int64_t i = cb + pr;
            if (pv < a.nv && i < ib) {
                int64_t o0, o1;
                if (i >= pw0 && i < pw1) {  // probed by the row search
                    o0 = s_po[i - pw0];
                    o1 = s_po[i - pw0 + 1];
                } else {
                    o0 = a.offs[i];
                    o1 = a.offs[i + 1];
                }
                o0 = o0 < 0 ? 0 : (o0 > a.nbytes ? a.nbytes : o0);
                o1 = o1 < o0 ? o0 : (o1 > a.nbytes ? a.nbytes : o1);
                ro0 = o0;
                ro1 = o1;
            }
        };
        load_offs(ia);
        if (PF) {
            pf = L + G < a.ntiles;
            if (pf) {
                const int64_t tn = xcd_tile(L + G, a.ntiles);  // this block's next tile
                probe_load(tn * B - a.shift);  // the search has moved this tile's probe to LDS
                probed = true;
                pf = tile_interior<U>(a, tn);
                if (pf) fetch_tile<U>(a, tn, v, halo, stid);
            }
        }
        for (int64_t cb = ia; cb < ib; cb += R) {
            if (cb != ia) load_offs(cb);
            const int nrc = (int)((ib - cb) < R ? (ib - cb) : R);  // rows in this chunk
            int64_t nint = 0, nedge = 0;  // this pair's interior and edge groups
            if (pv < a.nv && pr < nrc) {
                // segment of row i for vocabulary pv
                const int64_t i = cb + pr;
                const VocabLds &vl = vtab[pv];
                const int32_t k = KMER ? vl.k : 1;
                const Row r = make_row(ro0, ro1, k, vl.kinv);
                int64_t clo = 0, chi = 0;
                if (!(a.padded && r.len > vl.W)) {
                    clo = cells_before(r, P0, k, vl.kinv, a.cls, a.padded, a.left, vl.W);
                    chi = cells_before(r, P1, k, vl.kinv, a.cls, a.padded, a.left, vl.W);
                }
                const int64_t ncell = chi - clo;
                const int64_t lead = (a.padded && a.left) ? vl.W - r.len : 0;
                const int64_t tt0 = clo - lead;  // token index of the first owned cell
                SegInfo sg;
                sg.ncell = (int32_t)ncell;
                sg.b0 = clamp_cells(a.cls - tt0, ncell);
                sg.b1 = clamp_cells(a.cls + r.nb - tt0, ncell);
                sg.cc_cls = a.cls ? clamp_rel(-tt0, ncell) : -1;
                sg.cc_sep = a.cls ? clamp_rel(r.len - 1 - tt0, ncell) : -1;
                sg.cc_tail = (KMER && r.nb > 0 && r.nb * k != r.end - r.off) ? clamp_rel(a.cls + r.nb - 1 - tt0, ncell) : -1;
                sg.base_idx = (uint32_t)((r.off - P0) + (tt0 - a.cls) * k);
                sg.dlo = a.padded ? i * vl.W + clo : (a.fused_packed ? s_prefix[i] : vl.out_offs[i] - vl.base) + clo;
                const SegGroups gg =
                    seg_groups(sg.dlo, vl.al, sg.ncell, sg.b0, sg.b1, sg.cc_tail, a.padded != 0, vl.cap);
                nint = gg.gB - gg.gA;
                nedge = (gg.gA - gg.gfirst) + (gg.glast + 1 - gg.gB);
                seg[tid] = sg;
            }
            // Interior groups (bits 40 up: fewer than 2^20 in a chunk) and
            // edge groups (low 40 bits) of all pairs, vocabulary-major, in
            // one scan.
            constexpr int64_t kEdgeMask = (1ll << 40) - 1;
            int64_t tot;
            const int64_t pk = dev::block_excl_scan<NT>((nint << 40) | nedge, s_tmp, &tot);
            const int64_t epre = pk & kEdgeMask;
            s_ipre[tid] = (int32_t)(pk >> 40);
            if (pv < a.nv && pr < nrc) {
                seg[tid].ipre = (int32_t)(pk >> 40);
                seg[tid].epre = epre;
            }
            if (pv < a.nv && pr == 0) s_vg[pv] = epre;  // vocabulary v's edges are [s_vg[v], s_vg[v + 1])
            if (tid == 0) {
                s_vg[a.nv] = tot & kEdgeMask;
                s_itot = tot >> 40;
            }
            __syncthreads();

            // Interior groups: each wave takes a contiguous share of them,
            // segment by segment, with the segment's and its vocabulary's
            // facts uniform across the wave and four groups per lane in flight.
            {
                constexpr int NW = NT / dev::kWave;
                const int32_t T = (int32_t)s_itot;
                const int wv = tid / dev::kWave, lane = tid & (dev::kWave - 1);
                const int32_t x0 = (int32_t)((int64_t)T * wv / NW), x1 = (int32_t)((int64_t)T * (wv + 1) / NW);
                // the pair holding interior group x: the last one whose first
                // interior group is <= x (it holds at least one)
                auto pair_of = [&](int32_t x) {
                    int cnt = 0;
#pragma unroll
                    for (int r4 = 0; r4 < NT / dev::kWave; ++r4)
                        cnt += __popcll(__ballot(s_ipre[r4 * dev::kWave + lane] <= x));
                    return cnt - 1;
                };
                if (x0 < x1) {
                    int32_t x = x0;
                    while (x < x1) {
                        const int sidx = rfl(pair_of(x));
                        const int vi = rfl(sidx / R);
                        const VocabOut &o = a.vo[vi];
                        const int32_t k = KMER ? o.k : 1;
                        const int64_t al = o.al;
                        const SegInfo &sr = seg[sidx];
                        const int64_t dlo = rfl64(sr.dlo);
                        const uint32_t bidx = (uint32_t)rfl((int32_t)sr.base_idx);
                        const int32_t ipre = rfl(sr.ipre);
                        const SegGroups gg = seg_groups(dlo, al, rfl(sr.ncell), rfl(sr.b0), rfl(sr.b1), rfl(sr.cc_tail),
                                                        a.padded != 0, o.cap);
                        const int32_t n = (int32_t)(gg.gB - gg.gA);
                        const int32_t j0 = x - ipre;
                        const int32_t j1 = (x1 < ipre + n ? x1 : ipre + n) - ipre;
                        const int32_t cA = (int32_t)(4 * gg.gA - al - dlo);  // relative cell of group gA's first element
                        i32x4 *d4 = reinterpret_cast<i32x4 *>(o.ids + (4 * gg.gA - al));
                        int8_t *m1 = a.padded ? o.mask + (4 * gg.gA - al) : nullptr;  // PACKED has no mask
                        const bool mask4 = ((reinterpret_cast<uintptr_t>(o.mask) - (uintptr_t)al) & 3) == 0;
                        const bool k4 = k <= 8;
                        const Kmer4 kc = kmer4_consts(k4 ? k : 8);
                        auto ids_of = [&](int32_t j) {
                            const uint32_t idx0 = bidx + (uint32_t)(cA + 4 * j) * (uint32_t)k;
                            i32x4 y;
                            if (KMER && k4) {
                                y = kmer4_at(win64, val32, idx0, kc);
                            } else {
#pragma unroll
                                for (int rr = 0; rr < 4; ++rr) {
                                    const uint32_t idx = idx0 + (uint32_t)(rr * k);
                                    y[rr] = KMER ? kmer_at(win64, val32, idx, k) : lut_s[raw[idx]];
                                }
                            }
                            return y;
                        };
                        auto put = [&](int32_t j, i32x4 y) {
                            __builtin_nontemporal_store(y, d4 + j);
                            if (a.padded) {
                                if (mask4)
                                    *reinterpret_cast<uint32_t *>(m1 + 4 * j) = 0x01010101u;  // cached: L2 merges the words
                                else
                                    for (int rr = 0; rr < 4; ++rr) m1[4 * j + rr] = 1;
                            }
                        };
                        for (int32_t j = j0 + lane; j < j1; j += 4 * dev::kWave) {
                            const int32_t jb = j + dev::kWave, jc = j + 2 * dev::kWave, jd = j + 3 * dev::kWave;
                            const bool hb = jb < j1, hc = jc < j1, hd = jd < j1;
                            const i32x4 ya = ids_of(j);
                            const i32x4 yb = ids_of(hb ? jb : j);
                            const i32x4 yc = ids_of(hc ? jc : j);
                            const i32x4 yd = ids_of(hd ? jd : j);
                            put(j, ya);
                            if (hb) put(jb, yb);
                            if (hc) put(jc, yc);
                            if (hd) put(jd, yd);
                        }
                        x = ipre + j1;
                    }
                }
            }

            // Edge groups (CLS, SEP, short final frames, pads, ragged ends,
            // capacity overruns) cell by cell, vocabulary by vocabulary with
            // no barrier between them: edge q of vocabulary vi is written by
            // thread (q + 64 vi) % NT, so each vocabulary's edges start on
            // another wave and the vocabularies' dependent edge chains run
            // side by side (from one wave they took about 4 us per tile).
            for (int vi = 0; vi < a.nv; ++vi) {
                const VocabOut &o = a.vo[vi];
                const int32_t k = KMER ? o.k : 1;
                const int64_t al = o.al;
                int32_t *const ids_v = o.ids;
                int8_t *const mask_v = o.mask;
                const int64_t cap_v = o.cap;
                const bool mask4 = ((reinterpret_cast<uintptr_t>(mask_v) - (uintptr_t)al) & 3) == 0;
                const int64_t q0 = s_vg[vi], q1 = s_vg[vi + 1];
                const int sbase = vi * R;
                // cached segment: edges [seg_lo, seg_hi), head edges h of them
                int64_t seg_lo = 0, seg_hi = -1, gfirst = 0, gB = 0, h = 0;
                SegInfo sg{};
                for (int64_t qe = q0 + ((tid - dev::kWave * vi) & (NT - 1)); qe < q1; qe += NT) {
                    if (qe < seg_lo || qe >= seg_hi) {
                        int lo = sbase, hi = sbase + nrc - 1;
                        while (lo < hi) {  // last segment with epre <= qe
                            int mid = (lo + hi + 1) >> 1;
                            if (seg[mid].epre <= qe) lo = mid;
                            else hi = mid - 1;
                        }
                        sg = seg[lo];
                        seg_lo = sg.epre;
                        seg_hi = (lo + 1 < sbase + nrc) ? seg[lo + 1].epre : q1;
                        const SegGroups gg =
                            seg_groups(sg.dlo, al, sg.ncell, sg.b0, sg.b1, sg.cc_tail, a.padded != 0, cap_v);
                        gfirst = gg.gfirst;
                        gB = gg.gB;
                        h = gg.gA - gg.gfirst;
                    }
                    const int64_t le = qe - seg_lo;
                    const int64_t gq = le < h ? gfirst + le : gB + (le - h);
                    const int64_t eb = 4 * gq - al;
                    const int32_t cc0 = (int32_t)(eb - sg.dlo);
                    int32_t *dst = ids_v + eb;
                    int32_t vv[4];
                    uint32_t mk = 0;
                    bool in[4];
                    bool all_in = true;
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const int32_t cc = cc0 + rr;
                        in[rr] = (cc >= 0 && cc < sg.ncell);
                        if (in[rr] && !a.padded && (eb + rr < 0 || eb + rr >= cap_v)) {
                            in[rr] = false;
                            err |= DNATOK_DERR_CAPACITY;
                        }
                        all_in = all_in && in[rr];
                        int32_t val = o.pad_id;
                        uint32_t m = 0;
                        if (in[rr]) {
                            if (cc >= sg.b0 && cc < sg.b1) {
                                m = 1;
                                const uint32_t idx = sg.base_idx + (uint32_t)cc * (uint32_t)k;
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
                            int8_t *md = mask_v + eb;
                            if (mask4) {
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
                            if (a.padded) mask_v[eb + rr] = (int8_t)((mk >> (8 * rr)) & 1);
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    if (err) atomicOr(&s_err, err);
    __syncthreads();
    if (tid == 0 && s_err) dev::raise_error(a.err_hdr, s_err);
}

template <bool KMER, bool PF>
int launch_cells(const CellArgs &a, int U, int64_t grid, size_t dyn, hipStream_t stream) {
    switch (U) {
    case 1: hipLaunchKernelGGL((k_cells<KMER, 1, PF>), dim3((unsigned)grid), dim3(NT), dyn, stream, a); break;
    case 2: hipLaunchKernelGGL((k_cells<KMER, 2, PF>), dim3((unsigned)grid), dim3(NT), dyn, stream, a); break;
    case 4: hipLaunchKernelGGL((k_cells<KMER, 4, PF>), dim3((unsigned)grid), dim3(NT), dyn, stream, a); break;
    case 8: hipLaunchKernelGGL((k_cells<KMER, 8, PF>), dim3((unsigned)grid), dim3(NT), dyn, stream, a); break;
    case 16: hipLaunchKernelGGL((k_cells<KMER, 16, PF>), dim3((unsigned)grid), dim3(NT), dyn, stream, a); break;
    default: return set_error(DNATOK_EINVAL, "unsupported staging depth %d", U);
    }
    DNATOK_HIP(hipGetLastError());
    return DNATOK_OK;
}

template <bool KMER, bool PF>
int blocks_per_cu(int U, size_t dyn, int *out) {
    *out = 1;
    switch (U) {
    case 1: DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_cells<KMER, 1, PF>, NT, dyn)); break;
    case 2: DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_cells<KMER, 2, PF>, NT, dyn)); break;
    case 4: DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_cells<KMER, 4, PF>, NT, dyn)); break;
    case 8: DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_cells<KMER, 8, PF>, NT, dyn)); break;
    case 16: DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_cells<KMER, 16, PF>, NT, dyn)); break;
    default: break;
    }
    return DNATOK_OK;
}

}  // namespace

int launch_rowscan_spec(const RowScanSpec &sp, hipStream_t stream) {
    RowScanArgs s;
    s.offs = sp.offs;
    s.n = sp.n;
    s.nbytes = sp.nbytes;
    s.out_offs = sp.out;
    s.k = sp.k > 0 ? sp.k : 1;
    s.kinv = 0xFFFFFFFFu / (uint32_t)s.k;
    s.kmer = sp.kmer;
    s.overlap = sp.overlap;
    s.cls = sp.cls;
    s.padded = sp.padded;
    s.W = sp.W;
    s.base = sp.base;
    s.nunits = ((int64_t)sp.n + kUnitRows - 1) / kUnitRows;
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

int launch_rowscan(const int64_t *d_offsets, int32_t n, int64_t nbytes, int64_t *d_out, int32_t divisor, int32_t cls,
                   hipStream_t stream) {
    RowScanSpec sp;
    sp.offs = d_offsets;
    sp.n = n;
    sp.nbytes = nbytes;
    sp.out = d_out;
    sp.k = divisor;
    sp.kmer = 1;
    sp.overlap = 0;
    sp.cls = cls;
    sp.padded = 0;
    sp.W = 0;
    sp.base = 0;
    return launch_rowscan_spec(sp, stream);
}

EncodeTuning encode_tuning(const dnatok_vocab *v, int64_t nbytes) {
    const bool kmer = (v->kind == DNATOK_KMER);
    EncodeTuning t;
    const int32_t tile = v->tune_tile.load(std::memory_order_relaxed);
    if (tile > 0) {
        t.tile_bytes = tile;
    } else {
        // Untuned: 32 KiB (k-mer) or 16 KiB tiles, halved down to 4 KiB while
        // the batch would give fewer than two tiles per CU (a 1 Mbase batch
        // would otherwise run on a fraction of the chip).
        int64_t want = kmer ? 32768 : 16384;
        const int64_t target = nbytes / (2 * (int64_t)device_cu_count());
        while (want > 4096 && want > target) want >>= 1;
        t.tile_bytes = want;
    }
    t.blocks_per_cu = v->tune_blocks.load(std::memory_order_relaxed);
    t.spread = v->tune_spread.load(std::memory_order_relaxed);
    t.bands = v->tune_bands.load(std::memory_order_relaxed);
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
    const EncodeTuning tune = encode_tuning(v, nbytes);
    if (o.layout == DNATOK_PADDED && (tune.bands == 1 || tune.bands == 3)) {
        bool used = false;
        int rc = launch_encode_bands(vs, nv, d_bytes, nbytes, d_offsets, n, d_ids, caps, d_masks, os,
                                     tune.tile_bytes, tune.bands == 3, d_out_offsets, stream, &used);
        if (rc || used) return rc;
    }
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
        out.kinv = 0xFFFFFFFFu / (uint32_t)out.k;
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
        sc.kinv = out.kinv;
        sc.kmer = kmer ? 1 : 0;
        sc.overlap = 0;
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
    a.lut_off = (int32_t)dyn_tile;
    a.prefix_off = (int32_t)(dyn_tile + (kmer ? 0 : 1024));
    const size_t dyn = (size_t)a.prefix_off + (a.fused_packed ? 8 * (size_t)(n + 1) : 0);
    // As many tile walkers as fit, then evened out so every walker takes the
    // same number of tiles (no straggler round). Walkers with more than one
    // tile use the prefetching kernel, whose occupancy may be lower.
    int64_t per_block = 1;
    for (int pass = 0; pass < 2; ++pass) {
        const bool pfk = pass == 1;
        int per_cu = 0;
        rc = kmer ? (pfk ? blocks_per_cu<true, true>(U, dyn, &per_cu) : blocks_per_cu<true, false>(U, dyn, &per_cu))
                  : (pfk ? blocks_per_cu<false, true>(U, dyn, &per_cu) : blocks_per_cu<false, false>(U, dyn, &per_cu));
        if (rc) return rc;
        if (per_cu < 1) per_cu = 1;
        if (tune.blocks_per_cu > 0 && tune.blocks_per_cu < per_cu) per_cu = tune.blocks_per_cu;
        const int64_t gmax = (int64_t)device_cu_count() * per_cu;
        per_block = (a.ntiles + gmax - 1) / gmax;
        if (per_block == 1) break;  // one tile each: no prefetch
    }
    a.lead = 0;
    a.nstat = 0;
    a.nticket = 0;
    a.ticket = ws->d_hdr + HDR_TICKET;
    if (tune.spread > 0) {
        // One tile per workgroup: the first resident round by index, the
        // rest by ticket, plus spread% of the tiles as extra workgroups.
        // Workgroups go to the XCDs in turn whatever their speed, so extra
        // ones let an XCD that finishes early draw more of the tickets.
        int per_cu = 0;
        rc = kmer ? blocks_per_cu<true, false>(U, dyn, &per_cu) : blocks_per_cu<false, false>(U, dyn, &per_cu);
        if (rc) return rc;
        if (per_cu < 1) per_cu = 1;
        if (tune.blocks_per_cu > 0 && tune.blocks_per_cu < per_cu) per_cu = tune.blocks_per_cu;
        const int64_t resident = (int64_t)device_cu_count() * per_cu;
        if (a.ntiles > resident) {
            a.lead = a.fused_scan ? 8 : 0;  // keeps tile block b on XCD b % 8
            a.nstat = resident;
            a.nticket = (a.ntiles - resident) + (a.ntiles * tune.spread + 99) / 100;
            const int64_t grid = a.lead + a.nstat + a.nticket;
            return kmer ? launch_cells<true, false>(a, U, grid, dyn, stream)
                        : launch_cells<false, false>(a, U, grid, dyn, stream);
        }
    }
    const bool pf = per_block > 1;
    int64_t grid = (a.ntiles + per_block - 1) / per_block;
    if (a.fused_scan) grid += nv;
    if (kmer) return pf ? launch_cells<true, true>(a, U, grid, dyn, stream) : launch_cells<true, false>(a, U, grid, dyn, stream);
    return pf ? launch_cells<false, true>(a, U, grid, dyn, stream) : launch_cells<false, false>(a, U, grid, dyn, stream);
}

int launch_encode(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                  int32_t n, int32_t *d_ids, int64_t cap, int64_t *d_out_offsets, int8_t *d_mask,
                  const dnatok_encode_opts &o, hipStream_t stream) {
    return launch_encode_multi(&v, 1, d_bytes, nbytes, d_offsets, n, &d_ids, &cap, &d_out_offsets, &d_mask, &o,
                               stream);
}

}  // namespace dnatok
