// Output-parallel cell kernel: encode variants (reverse complement,
// overlapping k-mers) and the embedding lookup, fused with the encode or
// applied to given identifiers.
//
// Paper: Design (the embedder embed_tokens maps B x T identifiers to
// B x T x D activations; the bytes branch of the EmbedFromStrings algorithm
// maps bytes to identifiers on the device, left-pads them to token_len and
// hands them to embed_tokens); Discussion, "Integration with Data
// Augmentation" (reverse complement as a character-level map suited to the
// GPU); Introduction (overlapping k-mers of stride 1, L - k + 1 tokens).
//
// MI355X-first decomposition. In these forms the output dominates the
// traffic: an embedding row of D values per token (256 bytes for D = 128 in
// bf16, against about one input byte), or one id per base for stride-1
// windows. Work is therefore cut by output cells rather than input tiles:
//  * A block takes chunks of NT * CPT consecutive cells (cells = tokens plus
//    pads). Each thread works out the ids of CPT cells, NT apart so that id
//    and mask stores stay coalesced: the row a cell falls in (PADDED: cell /
//    W with a 32-bit reciprocal; PACKED: the chunk's first and last rows by
//    one-wave 64-way searches over the row starts the row scan wrote, then a
//    binary search between them), the token it holds (pad, CLS, SEP or a
//    body token), and the body token from the row's bytes.
//  * With an embedding table the chunk's ids go to LDS and the block copies
//    the table rows out in UB-byte units (UB = 16 whenever the row size and
//    pointers allow): lane l of a wave moves unit l, so a wave writes 1 KiB
//    of contiguous output per instruction. Several units are loaded before
//    any is stored. Table rows are read through L2 (a 4101 x 256-byte table
//    is 1 MiB, resident there); the output is the only HBM stream.
// Bounds: every output index is below the capacity the caller gave; bad
// offsets are clamped exactly as the row scan clamps them, so cell positions
// and the written offsets agree.
#include "common.hpp"
#include "device.hpp"

namespace dnatok {

namespace {

constexpr int NT = 256;
constexpr int CPT = 4;                       // cells per thread per chunk
constexpr int64_t kChunk = (int64_t)NT * CPT;
constexpr int kCopyUnroll = 4;               // table units loaded before they are stored

enum CwMode { CW_ENCODE = 0, CW_EMBED = 1, CW_GATHER = 2 };

struct CwArgs {
    const uint8_t *bytes;
    int64_t nbytes;
    const int64_t *offs;
    int32_t n;
    int32_t lut_kind;        // 1: id = lut[byte] (SINGLE, LUT256); 0: k-mer windows
    const int64_t *out_offs; // PACKED row starts (offset_base included)
    int64_t base;
    int64_t ncells;          // PADDED: n * W; GATHER: n_ids; PACKED: -1 (read out_offs[n])
    int64_t cap;             // cells the outputs hold
    int32_t k;
    int32_t stride;          // k (frames) or 1 (overlapping windows)
    int32_t overlap;
    int32_t revcomp;
    int32_t cls, padded, left;
    int64_t W;
    uint32_t winv;           // floor((2^32 - 1) / W) when W < 2^31, else 0
    int32_t pad_id, cls_id, sep_id;
    const int32_t *lut;
    int32_t *ids;            // optional for EMBED
    int8_t *mask;            // PADDED, optional for EMBED
    const int32_t *ids_in;   // GATHER
    const uint8_t *table;
    int64_t n_rows;
    int64_t row_bytes;
    uint8_t *emb;
    uint32_t ru, ruinv;      // units per table row and floor((2^32 - 1) / ru)
    uint32_t *err_hdr;
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <int UB>
struct Unit;
template <>
struct Unit<16> {
    typedef u32x4 T;
};
template <>
struct Unit<8> {
    typedef u32x2 T;
};
template <>
struct Unit<4> {
    typedef uint32_t T;
};
template <>
struct Unit<2> {
    typedef uint16_t T;
};
template <>
struct Unit<1> {
    typedef uint8_t T;
};

// x / d for x < 2^32 with dinv = floor((2^32 - 1) / d): the high product is
// the quotient or one less, and one step corrects it.
__device__ __forceinline__ uint32_t udiv(uint32_t x, uint32_t d, uint32_t dinv) {
    uint32_t q = __umulhi(x, dinv);
    if (x - q * d >= d) ++q;
    return q;
}

// Base digit A/a=0 C/c=1 G/g=2 T/t=3, or -1 for any other byte.
__device__ __forceinline__ int32_t base_digit(uint32_t b) {
    const uint32_t f = b | 0x20u;  // only 'A' and 'a' fold to 'a', and so on
    return f == 'a' ? 0 : f == 'c' ? 1 : f == 'g' ? 2 : f == 't' ? 3 : -1;
}

// Watson-Crick complement of a byte, case kept; other bytes unchanged.
__device__ __forceinline__ uint32_t complement(uint32_t b) {
    switch (b) {
    case 'A': return 'T';
    case 'T': return 'A';
    case 'C': return 'G';
    case 'G': return 'C';
    case 'a': return 't';
    case 't': return 'a';
    case 'c': return 'g';
    case 'g': return 'c';
    default: return b;
    }
}

// Row facts with offsets clamped as the row scan clamps them.
struct RowFacts {
    int64_t o0, o1, nb, len;
};

__device__ __forceinline__ RowFacts row_facts(const CwArgs &a, int64_t r) {
    RowFacts f;
    int64_t o0 = a.offs[r], o1 = a.offs[r + 1];
    o0 = o0 < 0 ? 0 : (o0 > a.nbytes ? a.nbytes : o0);
    o1 = o1 < o0 ? o0 : (o1 > a.nbytes ? a.nbytes : o1);
    const int64_t L = o1 - o0;
    int64_t nb;
    if (a.lut_kind) nb = L;
    else if (a.overlap) nb = L >= a.k ? L - a.k + 1 : (L > 0 ? 1 : 0);
    else nb = (L + a.k - 1) / a.k;
    f.o0 = o0;
    f.o1 = o1;
    f.nb = nb;
    f.len = nb + 2 * a.cls;
    return f;
}

// Id of body token j of a row (reverse complement: of the row read back to
// front with bases complemented).
__device__ __forceinline__ int32_t body_id(const CwArgs &a, const int32_t *s_lut, const RowFacts &f, int64_t j) {
    if (a.lut_kind) {
        const int64_t pos = a.revcomp ? f.o1 - 1 - j : f.o0 + j;
        uint32_t b = a.bytes[pos];
        if (a.revcomp) b = complement(b);
        return s_lut[b];
    }
    const int64_t s = j * a.stride;
    if (s + a.k > f.o1 - f.o0) return DNATOK_ID_UNK;  // short final frame, or a row shorter than k
    int32_t acc = 0;
    bool ok = true;
    for (int t = 0; t < a.k; ++t) {
        const int64_t pos = a.revcomp ? f.o1 - 1 - (s + t) : f.o0 + s + t;
        int32_t d = base_digit(a.bytes[pos]);
        ok = ok && d >= 0;
        if (a.revcomp) d = 3 - d;
        acc = acc * 4 + (d & 3);
    }
    return ok ? 5 + acc : DNATOK_ID_UNK;
}

// Id of position p of a row's span (PADDED: 0 <= p < W; PACKED: p < len).
__device__ __forceinline__ int32_t cell_id(const CwArgs &a, const int32_t *s_lut, const RowFacts &f, int64_t p,
                                           bool &tok) {
    int64_t q = p;
    if (a.padded && a.left) q = p - (a.W - f.len);
    tok = q >= 0 && q < f.len;
    if (!tok) return a.pad_id;
    if (a.cls) {
        if (q == 0) return a.cls_id;
        if (q == f.len - 1) return a.sep_id;
        return body_id(a, s_lut, f, q - 1);
    }
    return body_id(a, s_lut, f, q);
}

// Row of a PACKED cell: the first r with out_offs[r + 1] - base > cell.
__device__ __forceinline__ int64_t packed_row(const CwArgs &a, int64_t lo, int64_t hi, int64_t cell) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.out_offs[mid + 1] - a.base > cell) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

template <int MODE, int UB>
__global__ __launch_bounds__(NT) void k_cellwise(CwArgs a) {
    __shared__ int32_t s_lut[256];
    __shared__ int32_t s_id[kChunk];
    __shared__ int64_t s_rows[2];
    const int tid = threadIdx.x;
    if (MODE != CW_GATHER) s_lut[tid] = a.lut[tid];
    int64_t total = a.ncells;
    if (total < 0) total = a.out_offs[a.n] - a.base;
    const int64_t limit = total < a.cap ? total : a.cap;
    if (blockIdx.x == 0 && tid == 0 && total > a.cap) dev::raise_error(a.err_hdr, DNATOK_DERR_CAPACITY);
    uint32_t err = 0;
    __syncthreads();

    for (int64_t c0 = (int64_t)blockIdx.x * kChunk; c0 < limit; c0 += (int64_t)gridDim.x * kChunk) {
        const int64_t ncell = limit - c0 < kChunk ? limit - c0 : kChunk;
        if (MODE != CW_GATHER && !a.padded) {
            // the chunk's first and last rows, one wave each
            const int w = tid / dev::kWave;
            if (w < 2) {
                const int64_t key = w == 0 ? c0 : c0 + ncell - 1;
                const int64_t r = dev::wave_lower_bound(0, a.n, [&](int64_t q) { return a.out_offs[q + 1] - a.base > key; });
                if ((tid & (dev::kWave - 1)) == 0) s_rows[w] = r;
            }
            __syncthreads();
        }
        // row and position of this thread's first cell (PADDED)
        int64_t prow = 0, pp = 0;
        if (MODE != CW_GATHER && a.padded) {
            const int64_t c = c0 + tid;
            prow = c / a.W;
            pp = c - prow * a.W;
        }
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
            const int64_t d = (int64_t)tid + (int64_t)i * NT;
            const int64_t c = c0 + d;
            int32_t id = 0;
            if (d < ncell) {
                if (MODE == CW_GATHER) {
                    id = a.ids_in[c];
                    if (id < 0 || id >= a.n_rows) {
                        err |= DNATOK_DERR_IDS;
                        id = -1;
                    }
                } else {
                    bool tok;
                    if (a.padded) {
                        const RowFacts f = row_facts(a, prow);
                        id = cell_id(a, s_lut, f, pp, tok);
                        if (a.mask) a.mask[c] = tok ? 1 : 0;
                    } else {
                        const int64_t r = packed_row(a, s_rows[0], s_rows[1], c);
                        const RowFacts f = row_facts(a, r);
                        id = cell_id(a, s_lut, f, c - (a.out_offs[r] - a.base), tok);
                    }
                    if (a.ids) a.ids[c] = id;
                }
            }
            if (MODE != CW_ENCODE) s_id[d] = id;
            if (MODE != CW_GATHER && a.padded && i + 1 < CPT) {
                // advance to the cell NT further on
                pp += NT;
                if (a.winv) {
                    const uint32_t q = udiv((uint32_t)pp, (uint32_t)a.W, a.winv);
                    prow += q;
                    pp -= (int64_t)q * a.W;
                } else if (pp >= a.W) {
                    pp -= a.W;  // W >= 2^31 > NT: one row at most
                    ++prow;
                }
            }
        }
        if (MODE != CW_ENCODE) {
            typedef typename Unit<UB>::T V;
            __syncthreads();
            const uint32_t units = (uint32_t)ncell * a.ru;
            uint8_t *ob = a.emb + c0 * a.row_bytes;
            for (uint32_t u0 = tid; u0 < units; u0 += NT * kCopyUnroll) {
                V v[kCopyUnroll];
                uint32_t cell[kCopyUnroll], part[kCopyUnroll];
#pragma unroll
                for (int t = 0; t < kCopyUnroll; ++t) {
                    const uint32_t u = u0 + t * NT;
                    cell[t] = udiv(u, a.ru, a.ruinv);
                    part[t] = u - cell[t] * a.ru;
                    const int32_t id = u < units ? s_id[cell[t]] : -1;
                    if (id >= 0) v[t] = *reinterpret_cast<const V *>(a.table + (int64_t)id * a.row_bytes + part[t] * UB);
                    else v[t] = V{};
                }
#pragma unroll
                for (int t = 0; t < kCopyUnroll; ++t) {
                    const uint32_t u = u0 + t * NT;
                    if (u < units)
                        __builtin_nontemporal_store(v[t], reinterpret_cast<V *>(ob + (int64_t)cell[t] * a.row_bytes + part[t] * UB));
                }
            }
        }
        __syncthreads();
    }
    if (err) dev::raise_error(a.err_hdr, err);
}

template <int MODE, int UB>
int launch_cw(const CwArgs &a, int64_t max_cells, hipStream_t stream) {
    int per_cu = 0;
    DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cellwise<MODE, UB>, NT, 0));
    int64_t g = (int64_t)device_cu_count() * (per_cu > 0 ? per_cu : 1);
    const int64_t chunks = (max_cells + kChunk - 1) / kChunk;
    if (g > chunks) g = chunks;
    if (g < 1) g = 1;
    hipLaunchKernelGGL((k_cellwise<MODE, UB>), dim3((unsigned)g), dim3(NT), 0, stream, a);
    DNATOK_HIP(hipGetLastError());
    return DNATOK_OK;
}

template <int MODE>
int launch_cw_units(CwArgs &a, int64_t max_cells, hipStream_t stream) {
    // widest unit dividing the row size and both row bases
    const uintptr_t al = reinterpret_cast<uintptr_t>(a.table) | reinterpret_cast<uintptr_t>(a.emb) |
                         (uintptr_t)a.row_bytes;
    int ub = 16;
    while (ub > 1 && (al & (uintptr_t)(ub - 1))) ub >>= 1;
    a.ru = (uint32_t)(a.row_bytes / ub);
    a.ruinv = 0xFFFFFFFFu / a.ru;
    switch (ub) {
    case 16: return launch_cw<MODE, 16>(a, max_cells, stream);
    case 8: return launch_cw<MODE, 8>(a, max_cells, stream);
    case 4: return launch_cw<MODE, 4>(a, max_cells, stream);
    case 2: return launch_cw<MODE, 2>(a, max_cells, stream);
    default: return launch_cw<MODE, 1>(a, max_cells, stream);
    }
}

// Common set-up of the encode-side modes: row scan (out_offsets), then
// the cell arguments.
int setup_encode(CwArgs &a, const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                 int32_t n, int64_t *d_out_offsets, const dnatok_encode_opts &o, hipStream_t stream,
                 int64_t *max_cells) {
    const bool kmer = v->kind == DNATOK_KMER;
    a = CwArgs{};
    a.bytes = d_bytes;
    a.nbytes = nbytes;
    a.offs = d_offsets;
    a.n = n;
    a.lut_kind = kmer ? 0 : 1;
    a.out_offs = d_out_offsets;
    a.base = o.offset_base;
    a.k = kmer ? v->k : 1;
    a.overlap = (o.variant & DNATOK_VARIANT_OVERLAP) ? 1 : 0;
    a.stride = a.overlap ? 1 : a.k;
    a.revcomp = (o.variant & DNATOK_VARIANT_REVCOMP) ? 1 : 0;
    a.cls = o.add_cls_sep ? 1 : 0;
    a.padded = o.layout == DNATOK_PADDED ? 1 : 0;
    a.left = o.pad_side == DNATOK_PAD_LEFT ? 1 : 0;
    a.W = a.padded ? o.pad_to : 0;
    a.winv = (a.padded && a.W < ((int64_t)1 << 31)) ? 0xFFFFFFFFu / (uint32_t)a.W : 0;
    a.pad_id = v->pad_id;
    a.cls_id = v->cls_id;
    a.sep_id = v->sep_id;
    a.lut = v->d_lut;

    RowScanSpec sp;
    sp.offs = d_offsets;
    sp.n = n;
    sp.nbytes = nbytes;
    sp.out = d_out_offsets;
    sp.k = a.k;
    sp.kmer = kmer ? 1 : 0;
    sp.overlap = a.overlap;
    sp.cls = a.cls;
    sp.padded = a.padded;
    sp.W = a.W;
    sp.base = a.base;
    int rc = launch_rowscan_spec(sp, stream);
    if (rc) return rc;
    Workspace *ws = nullptr;
    rc = get_workspace(stream, 1, &ws);
    if (rc) return rc;
    a.err_hdr = ws->d_hdr;
    a.ncells = a.padded ? (int64_t)n * a.W : -1;
    *max_cells = a.padded ? a.ncells : -1;
    return DNATOK_OK;
}

}  // namespace

int launch_encode_variant(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                          int32_t n, int32_t *d_ids, int64_t cap, int64_t *d_out_offsets, int8_t *d_mask,
                          const dnatok_encode_opts &o, hipStream_t stream) {
    CwArgs a;
    int64_t max_cells = 0;
    int rc = setup_encode(a, v, d_bytes, nbytes, d_offsets, n, d_out_offsets, o, stream, &max_cells);
    if (rc) return rc;
    a.ids = d_ids;
    a.mask = a.padded ? d_mask : nullptr;
    a.cap = cap;
    if (max_cells < 0 || max_cells > cap) max_cells = cap;
    return launch_cw<CW_ENCODE, 16>(a, max_cells, stream);
}

int launch_embed(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets, int32_t n,
                 const void *d_table, int64_t n_rows, int64_t row_bytes, void *d_out, int64_t out_rows,
                 int64_t *d_out_offsets, int32_t *d_ids, int8_t *d_mask, const dnatok_encode_opts &o,
                 hipStream_t stream) {
    CwArgs a;
    int64_t max_cells = 0;
    int rc = setup_encode(a, v, d_bytes, nbytes, d_offsets, n, d_out_offsets, o, stream, &max_cells);
    if (rc) return rc;
    a.ids = d_ids;
    a.mask = a.padded ? d_mask : nullptr;
    a.cap = out_rows;
    a.table = static_cast<const uint8_t *>(d_table);
    a.n_rows = n_rows;
    a.row_bytes = row_bytes;
    a.emb = static_cast<uint8_t *>(d_out);
    if (max_cells < 0 || max_cells > out_rows) max_cells = out_rows;
    return launch_cw_units<CW_EMBED>(a, max_cells, stream);
}

int launch_embed_ids(const int32_t *d_ids, int64_t n_ids, const void *d_table, int64_t n_rows, int64_t row_bytes,
                     void *d_out, hipStream_t stream) {
    CwArgs a = CwArgs{};
    Workspace *ws = nullptr;
    int rc = get_workspace(stream, 1, &ws);
    if (rc) return rc;
    a.err_hdr = ws->d_hdr;
    a.ids_in = d_ids;
    a.ncells = n_ids;
    a.cap = n_ids;
    a.table = static_cast<const uint8_t *>(d_table);
    a.n_rows = n_rows;
    a.row_bytes = row_bytes;
    a.emb = static_cast<uint8_t *>(d_out);
    return launch_cw_units<CW_GATHER>(a, n_ids, stream);
}

}  // namespace dnatok
