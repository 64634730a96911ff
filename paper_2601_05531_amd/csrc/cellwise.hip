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
//    pads); each thread takes CPT consecutive cells of the chunk, so its ids
//    go out as one 16-byte store and its mask bytes as one word. The thread
//    finds the row of its first cell (PADDED: cell / W with a 32-bit
//    reciprocal; PACKED: the chunk's first and last rows by one-wave 64-way
//    searches over the row starts the row scan wrote, then a binary search
//    between them) and steps to the next row only at a row end. It places
//    every cell first (pad, CLS, SEP or body token, and the bytes a body
//    token reads), then issues all of its reads at once: a k-mer reads the
//    three (k <= 8) or five dwords that hold it and classifies them with
//    the same 16-byte classifier the tile kernel uses; reverse complement
//    reverses and complements the digits in registers (the bytes are never
//    rewritten), and for table kinds it reads a table already mapped
//    through the complement.
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
#include "rowscan.hpp"

namespace dnatok {

namespace {

constexpr int NT = 256;
static_assert(NT == kScanNT, "the fused row scan runs with the cell kernel's block size");
constexpr int32_t kFuseMaxRows = 16384;      // PADDED: the first block scans the rows instead of a separate launch
constexpr int kGridPerSlot = 4;              // blocks launched per resident block slot
constexpr int CPT = 4;                       // cells per thread per chunk (a multiple of 4)
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
    uint32_t kinv;           // floor((2^32 - 1) / k)
    int32_t pad_id, cls_id, sep_id;
    const int32_t *lut;
    int32_t *ids;            // optional for EMBED
    int8_t *mask;            // PADDED, optional for EMBED
    const int32_t *ids_in;   // GATHER: int32 ids (or)
    const int64_t *ids_in64; // GATHER: int64 ids
    const uint8_t *table;
    int64_t n_rows;
    int64_t row_bytes;
    uint8_t *emb;
    uint32_t ru, ruinv;      // units per table row and floor((2^32 - 1) / ru)
    uint32_t *err_hdr;
    int32_t fused_scan;      // PADDED, few rows: block 0 writes out_offsets (the others take cells)
    RowScanArgs scan;
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

// x / d for x >= 0, d >= 1, with the 32-bit path when both fit.
__device__ __forceinline__ int64_t div_any(int64_t x, int64_t d, uint32_t dinv) {
    if (dinv && x < ((int64_t)1 << 32)) return udiv((uint32_t)x, (uint32_t)d, dinv);
    return x / d;
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
    else nb = div_any(L + a.k - 1, a.k, a.kinv);
    f.o0 = o0;
    f.o1 = o1;
    f.nb = nb;
    f.len = nb + 2 * a.cls;
    return f;
}

// The 16 bytes from p on, for a k-mer at p (k <= 8 needs three dwords,
// k <= 15 five). Dword addresses are clamped to the dword that holds the
// k-mer's last byte, so every read stays within the dwords the k-mer
// occupies; bytes past the k-mer are don't-cares.
template <bool K8>
__device__ __forceinline__ uint4 window16(const uint8_t *p, int32_t k) {
    constexpr int ND = K8 ? 3 : 5;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(p);
    const uint32_t sh = (uint32_t)(addr & 3);
    const uint8_t *first = p - sh;
    const uint8_t *last = p + (k - 1) - ((addr + (uintptr_t)(k - 1)) & 3);
    uint32_t w[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        if (i < ND) {
            const uint8_t *q = first + 4 * i;
            w[i] = *reinterpret_cast<const uint32_t *>(q < last ? q : last);
        } else {
            w[i] = 0;
        }
    }
    uint4 r;
    r.x = __builtin_amdgcn_alignbyte(w[1], w[0], sh);
    r.y = __builtin_amdgcn_alignbyte(w[2], w[1], sh);
    r.z = __builtin_amdgcn_alignbyte(w[3], w[2], sh);
    r.w = __builtin_amdgcn_alignbyte(w[4], w[3], sh);
    return r;
}

// Id of the k-mer whose bytes (in memory order) open window v; reverse
// complement: of those bytes taken back to front, each complemented.
__device__ __forceinline__ int32_t kmer_id(uint4 v, int32_t k, int32_t revcomp) {
    uint32_t code, valid;
    dev::classify16(v, code, valid);
    const uint32_t km = (1u << k) - 1u;
    if ((valid >> (32 - k)) != km) return DNATOK_ID_UNK;
    uint32_t x = code >> (32 - 2 * k);
    if (revcomp) {
        // digits in reverse order (bit reversal, then each 2-bit digit's
        // bits swapped back), each complemented (3 - d = d ^ 3)
        uint32_t y = __builtin_bitreverse32(x);
        y = ((y >> 1) & 0x55555555u) | ((y & 0x55555555u) << 1);
        x = (y >> (32 - 2 * k)) ^ ((1u << (2 * k)) - 1u);
    }
    return (int32_t)(5 + x);
}

// Row of a PACKED cell: the first r in [lo, hi] with out_offs[r + 1] - base > cell.
__device__ __forceinline__ int64_t packed_row(const CwArgs &a, int64_t lo, int64_t hi, int64_t cell) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.out_offs[mid + 1] - a.base > cell) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// Ids of the cells cb .. cb + CPT - 1 (those below cend) and whether each
// holds a token (not a pad). First every cell is placed (row, token kind,
// and for a body token the bytes it reads; other cells point their reads
// at the offsets array, which always holds a readable word), then all
// reads are issued, then the ids are formed. Rows change within a thread's
// cells only at row ends.
template <bool K8>
__device__ __forceinline__ void thread_cells(const CwArgs &a, const int32_t *s_lut, int64_t cb, int64_t cend,
                                             const int64_t *s_rows, int32_t (&id)[CPT], bool (&tok)[CPT]) {
    int64_t row, p;
    if (a.padded) {
        row = div_any(cb, a.W, a.winv);
        p = cb - row * a.W;
    } else {
        row = packed_row(a, s_rows[0], s_rows[1], cb);
        p = cb - (a.out_offs[row] - a.base);
    }
    RowFacts f = row_facts(a, row);
    // Fast path: the CPT cells are body tokens of this row whose windows
    // lie within 32 bytes (any overlapping k, frames of k <= 8, table
    // kinds): one 32-byte read, two classifications, then shifts per cell.
    {
        const int32_t kw = a.lut_kind ? 1 : a.k;
        const int32_t st = a.lut_kind ? 1 : a.stride;
        const int32_t spanb = (CPT - 1) * st + kw;
        int64_t q0 = p;
        if (a.padded && a.left) q0 = p - (a.W - f.len);
        const int64_t j0 = q0 - a.cls;
        const int64_t s0 = j0 * st;
        if (spanb <= 32 && cb + CPT <= cend && p + CPT <= (a.padded ? a.W : f.len) && q0 >= a.cls &&
            q0 + CPT <= f.len - a.cls && s0 + spanb <= f.o1 - f.o0) {
            const int64_t lo = a.revcomp ? f.o1 - s0 - spanb : f.o0 + s0;
            const uint8_t *pl = a.bytes + lo;
            const uintptr_t addr = reinterpret_cast<uintptr_t>(pl);
            const uint32_t sh = (uint32_t)(addr & 3);
            const uint8_t *first = pl - sh;
            const uint8_t *last = pl + (spanb - 1) - ((addr + (uintptr_t)(spanb - 1)) & 3);
            uint32_t w[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const uint8_t *q = first + 4 * i;
                w[i] = *reinterpret_cast<const uint32_t *>(q < last ? q : last);
            }
            if (a.lut_kind) {
                const uint32_t b4 = __builtin_amdgcn_alignbyte(w[1], w[0], sh);
#pragma unroll
                for (int i = 0; i < CPT; ++i) {
                    const int t = a.revcomp ? CPT - 1 - i : i;
                    id[i] = s_lut[(b4 >> (8 * t)) & 255u];
                    tok[i] = true;
                }
                return;
            }
            uint4 v0, v1;
            v0.x = __builtin_amdgcn_alignbyte(w[1], w[0], sh);
            v0.y = __builtin_amdgcn_alignbyte(w[2], w[1], sh);
            v0.z = __builtin_amdgcn_alignbyte(w[3], w[2], sh);
            v0.w = __builtin_amdgcn_alignbyte(w[4], w[3], sh);
            v1.x = __builtin_amdgcn_alignbyte(w[5], w[4], sh);
            v1.y = __builtin_amdgcn_alignbyte(w[6], w[5], sh);
            v1.z = __builtin_amdgcn_alignbyte(w[7], w[6], sh);
            v1.w = __builtin_amdgcn_alignbyte(w[8], w[7], sh);
            uint32_t c0, c1, va0, va1;
            dev::classify16(v0, c0, va0);
            dev::classify16(v1, c1, va1);
            const uint64_t code = ((uint64_t)c0 << 32) | c1;  // 32 digits, first byte on top
            const uint32_t valid = va0 | (va1 >> 16);         // 32 validity bits, first byte on top
            const int32_t k = a.k;
            const uint32_t km = (1u << k) - 1u;
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
                const int32_t off = (a.revcomp ? CPT - 1 - i : i) * st;  // window of cell i within the 32 bytes
                uint32_t x = (uint32_t)((code << (2 * off)) >> (64 - 2 * k));
                const bool ok = ((valid << off) >> (32 - k)) == km;
                if (a.revcomp) {
                    uint32_t y = __builtin_bitreverse32(x);
                    y = ((y >> 1) & 0x55555555u) | ((y & 0x55555555u) << 1);
                    x = (y >> (32 - 2 * k)) ^ ((1u << (2 * k)) - 1u);
                }
                id[i] = ok ? (int32_t)(5 + x) : DNATOK_ID_UNK;
                tok[i] = true;
            }
            return;
        }
    }
    const uint8_t *dummy = reinterpret_cast<const uint8_t *>(a.offs);
    const uint8_t *src[CPT];
    int32_t fixed[CPT], kk[CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        src[i] = dummy;
        fixed[i] = a.pad_id;
        kk[i] = 1;
        tok[i] = false;
        if (cb + i < cend) {
            if (p == (a.padded ? a.W : f.len)) {
                // the next row (PACKED: the next non-empty one; one exists,
                // since this cell is below the total)
                p = 0;
                do {
                    ++row;
                    f = row_facts(a, row);
                } while (!a.padded && f.len == 0);
            }
            int64_t q = p;
            if (a.padded && a.left) q = p - (a.W - f.len);
            tok[i] = q >= 0 && q < f.len;
            if (tok[i]) {
                if (a.cls && q == 0) {
                    fixed[i] = a.cls_id;
                } else if (a.cls && q == f.len - 1) {
                    fixed[i] = a.sep_id;
                } else {
                    const int64_t j = q - a.cls;
                    if (a.lut_kind) {
                        src[i] = a.bytes + (a.revcomp ? f.o1 - 1 - j : f.o0 + j);
                        fixed[i] = -1;
                    } else {
                        const int64_t s0 = j * a.stride;
                        if (s0 + a.k > f.o1 - f.o0) {
                            fixed[i] = DNATOK_ID_UNK;  // short final frame, or a row shorter than k
                        } else {
                            src[i] = a.bytes + (a.revcomp ? f.o1 - s0 - a.k : f.o0 + s0);
                            fixed[i] = -1;
                            kk[i] = a.k;
                        }
                    }
                }
            }
            ++p;
        }
    }
    if (a.lut_kind) {
        uint32_t b[CPT];
#pragma unroll
        for (int i = 0; i < CPT; ++i) b[i] = *src[i];
#pragma unroll
        for (int i = 0; i < CPT; ++i) id[i] = fixed[i] >= 0 ? fixed[i] : s_lut[b[i]];
    } else {
        uint4 win[CPT];
#pragma unroll
        for (int i = 0; i < CPT; ++i) win[i] = window16<K8>(src[i], kk[i]);
#pragma unroll
        for (int i = 0; i < CPT; ++i) id[i] = fixed[i] >= 0 ? fixed[i] : kmer_id(win[i], a.k, a.revcomp);
    }
}

template <int MODE, int UB, bool K8>
__global__ __launch_bounds__(NT) void k_cellwise(CwArgs a) {
    __shared__ int32_t s_lut[256];
    __shared__ int32_t s_id[kChunk];
    __shared__ int64_t s_rows[2];
    const int tid = threadIdx.x;
    if (MODE != CW_GATHER && a.fused_scan && blockIdx.x == 0) {
        __shared__ int64_t s_tmp[kScanNT / dev::kWave + 1];
        rowscan_single_block(a.scan, s_tmp, a.err_hdr);
        return;
    }
    const int64_t bid = (int64_t)blockIdx.x - a.fused_scan;  // cell walker index
    const int64_t G = (int64_t)gridDim.x - a.fused_scan;     // cell walkers
    if (MODE != CW_GATHER) s_lut[tid] = a.lut[a.revcomp ? complement((uint32_t)tid) : (uint32_t)tid];
    int64_t total = a.ncells;
    if (total < 0) total = a.out_offs[a.n] - a.base;
    const int64_t limit = total < a.cap ? total : a.cap;
    if (bid == 0 && tid == 0 && total > a.cap) dev::raise_error(a.err_hdr, DNATOK_DERR_CAPACITY);
    uint32_t err = 0;
    __syncthreads();

    for (int64_t c0 = bid * kChunk; c0 < limit; c0 += G * kChunk) {
        const int64_t cend = limit - c0 < kChunk ? limit : c0 + kChunk;
        if (MODE != CW_GATHER && !a.padded) {
            // the chunk's first and last rows, one wave each
            const int w = tid / dev::kWave;
            if (w < 2) {
                const int64_t key = w == 0 ? c0 : cend - 1;
                const int64_t r = dev::wave_lower_bound(0, a.n, [&](int64_t q) { return a.out_offs[q + 1] - a.base > key; });
                if ((tid & (dev::kWave - 1)) == 0) s_rows[w] = r;
            }
            __syncthreads();
        }
        // this thread's CPT consecutive cells
        const int64_t cb = c0 + (int64_t)tid * CPT;
        int32_t id[CPT];
        bool tok[CPT];
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
            id[i] = 0;
            tok[i] = false;
        }
        if (MODE == CW_GATHER) {
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
                if (cb + i < cend) {
                    const int64_t x = a.ids_in64 ? a.ids_in64[cb + i] : (int64_t)a.ids_in[cb + i];
                    id[i] = (int32_t)x;
                    if (x < 0 || x >= a.n_rows) {
                        err |= DNATOK_DERR_IDS;
                        id[i] = -1;
                    }
                }
            }
        } else if (cb < cend) {
            thread_cells<K8>(a, s_lut, cb, cend, s_rows, id, tok);
        }
        if (MODE != CW_GATHER && cb < cend) {
            const bool full = cb + CPT <= cend;
            if (a.ids) {
                if (full && ((reinterpret_cast<uintptr_t>(a.ids + cb) & 15) == 0)) {
#pragma unroll
                    for (int g = 0; g < CPT; g += 4)
                        *reinterpret_cast<int4 *>(a.ids + cb + g) = make_int4(id[g], id[g + 1], id[g + 2], id[g + 3]);
                } else {
#pragma unroll
                    for (int i = 0; i < CPT; ++i)
                        if (cb + i < cend) a.ids[cb + i] = id[i];
                }
            }
            if (a.mask) {
                if (full && ((reinterpret_cast<uintptr_t>(a.mask + cb) & 3) == 0)) {
#pragma unroll
                    for (int g = 0; g < CPT; g += 4)
                        *reinterpret_cast<uint32_t *>(a.mask + cb + g) = (uint32_t)tok[g] | (uint32_t)tok[g + 1] << 8 |
                                                                         (uint32_t)tok[g + 2] << 16 |
                                                                         (uint32_t)tok[g + 3] << 24;
                } else {
#pragma unroll
                    for (int i = 0; i < CPT; ++i)
                        if (cb + i < cend) a.mask[cb + i] = tok[i] ? 1 : 0;
                }
            }
        }
        if (MODE != CW_ENCODE) {
#pragma unroll
            for (int i = 0; i < CPT; ++i) s_id[tid * CPT + i] = id[i];
            typedef typename Unit<UB>::T V;
            __syncthreads();
            const uint32_t units = (uint32_t)(cend - c0) * a.ru;
            uint8_t *ob = a.emb + c0 * a.row_bytes;
            for (uint32_t u0 = tid; u0 < units; u0 += NT * kCopyUnroll) {
                V v[kCopyUnroll];
                uint32_t cell[kCopyUnroll], part[kCopyUnroll];
#pragma unroll
                for (int t = 0; t < kCopyUnroll; ++t) {
                    const uint32_t u = u0 + t * NT;
                    cell[t] = udiv(u, a.ru, a.ruinv);
                    part[t] = u - cell[t] * a.ru;
                    const int32_t rid = u < units ? s_id[cell[t]] : -1;
                    if (rid >= 0) v[t] = *reinterpret_cast<const V *>(a.table + (int64_t)rid * a.row_bytes + part[t] * UB);
                    else v[t] = V{};
                }
#pragma unroll
                for (int t = 0; t < kCopyUnroll; ++t) {
                    const uint32_t u = u0 + t * NT;
                    if (u < units)
                        __builtin_nontemporal_store(v[t], reinterpret_cast<V *>(ob + (int64_t)cell[t] * a.row_bytes + part[t] * UB));
                }
            }
            __syncthreads();
        } else if (!a.padded) {
            __syncthreads();  // s_rows is rewritten for the next chunk
        }
    }
    if (err) dev::raise_error(a.err_hdr, err);
}

template <int MODE, int UB, bool K8>
int launch_cw(const CwArgs &a, int64_t max_cells, hipStream_t stream) {
    int per_cu = 0;
    DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cellwise<MODE, UB, K8>, NT, 0));
    // several blocks per resident slot: a block that ends need not wait for
    // its stores, where a walker's next chunk would
    int64_t g = kGridPerSlot * (int64_t)device_cu_count() * (per_cu > 0 ? per_cu : 1);
    const int64_t chunks = (max_cells + kChunk - 1) / kChunk;
    if (g > chunks) g = chunks;
    if (g < 1) g = 1;
    g += a.fused_scan;
    hipLaunchKernelGGL((k_cellwise<MODE, UB, K8>), dim3((unsigned)g), dim3(NT), 0, stream, a);
    DNATOK_HIP(hipGetLastError());
    return DNATOK_OK;
}

// k-mers of up to 8 bases read three dwords per token, longer ones five.
template <int MODE, int UB>
int launch_cw_k(const CwArgs &a, int64_t max_cells, hipStream_t stream) {
    if (a.lut_kind || a.k <= 8) return launch_cw<MODE, UB, true>(a, max_cells, stream);
    return launch_cw<MODE, UB, false>(a, max_cells, stream);
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
    case 16: return launch_cw_k<MODE, 16>(a, max_cells, stream);
    case 8: return launch_cw_k<MODE, 8>(a, max_cells, stream);
    case 4: return launch_cw_k<MODE, 4>(a, max_cells, stream);
    case 2: return launch_cw_k<MODE, 2>(a, max_cells, stream);
    default: return launch_cw_k<MODE, 1>(a, max_cells, stream);
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
    a.kinv = 0xFFFFFFFFu / (uint32_t)a.k;
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

    Workspace *ws = nullptr;
    int rc = get_workspace(stream, 1, &ws);
    if (rc) return rc;
    a.fused_scan = (a.padded && n <= kFuseMaxRows) ? 1 : 0;
    if (a.fused_scan) {
        RowScanArgs &sc = a.scan;
        sc = RowScanArgs{};
        sc.offs = d_offsets;
        sc.n = n;
        sc.nbytes = nbytes;
        sc.out_offs = d_out_offsets;
        sc.k = a.k;
        sc.kinv = a.kinv;
        sc.kmer = kmer ? 1 : 0;
        sc.overlap = a.overlap;
        sc.cls = a.cls;
        sc.padded = 1;
        sc.W = a.W;
        sc.base = a.base;
    } else {
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
        rc = launch_rowscan_spec(sp, stream);
        if (rc) return rc;
    }
    a.err_hdr = ws->d_hdr;
    a.ncells = a.padded ? (int64_t)n * a.W : -1;
    *max_cells = a.padded ? a.ncells : -1;
    return DNATOK_OK;
}

}  // namespace

int launch_encode_variant(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                          int32_t n, int32_t *d_ids, int64_t cap, int64_t *d_out_offsets, int8_t *d_mask,
                          const dnatok_encode_opts &o, hipStream_t stream) {
    const EncodeTuning tune = encode_tuning(v, nbytes);
    if (o.layout == DNATOK_PADDED && (tune.bands == 1 || tune.bands == 3)) {
        bool used = false;
        int rc = launch_encode_bands(&v, 1, d_bytes, nbytes, d_offsets, n, &d_ids, &cap, &d_mask, &o,
                                     tune.tile_bytes, tune.bands == 3, &d_out_offsets, stream, &used);
        if (rc || used) return rc;
    }
    CwArgs a;
    int64_t max_cells = 0;
    int rc = setup_encode(a, v, d_bytes, nbytes, d_offsets, n, d_out_offsets, o, stream, &max_cells);
    if (rc) return rc;
    a.ids = d_ids;
    a.mask = a.padded ? d_mask : nullptr;
    a.cap = cap;
    if (max_cells < 0 || max_cells > cap) max_cells = cap;
    return launch_cw_k<CW_ENCODE, 16>(a, max_cells, stream);
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

int launch_embed_ids(const int32_t *d_ids, const int64_t *d_ids64, int64_t n_ids, const void *d_table,
                     int64_t n_rows, int64_t row_bytes, void *d_out, hipStream_t stream) {
    CwArgs a = CwArgs{};
    Workspace *ws = nullptr;
    int rc = get_workspace(stream, 1, &ws);
    if (rc) return rc;
    a.err_hdr = ws->d_hdr;
    a.ids_in = d_ids;
    a.ids_in64 = d_ids64;
    a.ncells = n_ids;
    a.cap = n_ids;
    a.table = static_cast<const uint8_t *>(d_table);
    a.n_rows = n_rows;
    a.row_bytes = row_bytes;
    a.emb = static_cast<uint8_t *>(d_out);
    return launch_cw_units<CW_GATHER>(a, n_ids, stream);
}

}  // namespace dnatok
