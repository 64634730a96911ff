// Decode: ids -> uppercase bases (the inverse table the paper lists as
// future work, Discussion, "Decode Operations": the same LUT principle run
// backwards). Not on the hot path.
//
// Tiles of TT token positions, each tile's output bytes contiguous. Two
// launches: a row pass (each tile's first row, the offsets check, and the
// tile status words cleared), then one workgroup per tile that reads its
// ids once, sums its output bytes, takes its output position by a
// decoupled look-back over the tiles before it (Merrill and Garland's
// single-pass prefix scan), stages its bytes in LDS at their 16-byte phase
// in the output and writes them with 16-byte stores. Tiles follow the
// workgroup index: a workgroup starts only after every lower-indexed one
// on its XCD, and the XCDs take workgroups in index order, so the tile
// with the lowest index still running never waits and the look-back ends
// (with no ticket counter: one device-wide counter serializes at about
// 12 ns per ticket, which at thousands of tiles outweighs the decode).
#include "common.hpp"
#include "device.hpp"

namespace dnatok {

namespace {

constexpr int NT = 256;
constexpr int TPT = 16;  // tokens per thread (fewer, smaller tiles measured slower for every kind)
constexpr int TT = NT * TPT;
constexpr int kMaxStage = 32768;
constexpr int TPT_SINGLE = 32;  // single-nucleotide ids per thread in the strided kernel
constexpr int TT_SINGLE = NT * TPT_SINGLE;  // most bytes of one tile's output staged in LDS

struct DecodeArgs {
    const int32_t *ids;
    int64_t n_ids;
    const int64_t *offs;
    int32_t n;
    uint8_t *out;
    int64_t cap;
    int64_t *out_offs;
    int32_t kind;
    int32_t k;
    int32_t vocab;
    const int32_t *tok_len;
    const int64_t *tok_off;
    const uint8_t *tok_chars;
    int64_t ntiles;
    int64_t tt;          // token positions per tile (TT, or TT_SINGLE for the strided single-nucleotide kernel)
    int32_t stage;       // bytes the LDS stage holds (a tile with more output writes its tokens directly)
    uint64_t *status;    // tile status words of the look-back (ntiles), cleared by the row pass
    int64_t *first_row;  // first row starting at or after each tile's first position (ntiles + 1)
    uint32_t *err_hdr;
};

__device__ __forceinline__ bool is_silent(int32_t id) {
    return id == DNATOK_ID_PAD || id == DNATOK_ID_CLS || id == DNATOK_ID_SEP || id == DNATOK_ID_MASK;
}

// Output bytes of one id. KIND is the vocabulary kind (a template
// parameter, so each kind's kernel holds only its own branch).
template <int KIND>
__device__ __forceinline__ int32_t width_of(const DecodeArgs &a, int32_t id) {
    if (is_silent(id)) return 0;
    if (KIND == DNATOK_KMER) return a.k;
    if (KIND == DNATOK_BPE && id >= 10 && id < a.vocab) return a.tok_len[id];
    return 1;
}

// The letter of 2-bit code c (0..3: A, C, G, T) from one packed word: a
// table in memory would cost a dependent load per base.
__device__ __forceinline__ uint8_t base_letter(uint32_t c) { return (uint8_t)(0x54474341u >> (8 * (c & 3))); }

// The letter of a single-nucleotide id (N and unknown ids: 'N').
__device__ __forceinline__ uint8_t single_letter(int32_t id) {
    return (id >= 5 && id <= 8) ? base_letter((uint32_t)(id - 5)) : (uint8_t)'N';
}

template <int KIND>
__device__ __forceinline__ void write_token(const DecodeArgs &a, int32_t id, int64_t pos, uint32_t &err) {
    if (is_silent(id)) return;
    if (KIND == DNATOK_KMER) {
        const bool known = id >= 5 && id < a.vocab;
        uint32_t v = known ? (uint32_t)(id - 5) : 0u;
#pragma unroll 1
        for (int j = a.k - 1; j >= 0; --j) {
            int64_t p = pos + j;
            if (p < a.cap) a.out[p] = known ? base_letter(v) : (uint8_t)'N';
            else err |= DNATOK_DERR_CAPACITY;
            v >>= 2;
        }
        return;
    }
    if (KIND == DNATOK_BPE && id >= 10 && id < a.vocab) {
        const int64_t L = a.tok_len[id], o = a.tok_off[id];
#pragma unroll 1
        for (int64_t j = 0; j < L; ++j) {
            if (pos + j < a.cap) a.out[pos + j] = a.tok_chars[o + j];
            else err |= DNATOK_DERR_CAPACITY;
        }
        return;
    }
    if (pos < a.cap) a.out[pos] = single_letter(id);
    else err |= DNATOK_DERR_CAPACITY;
}

// The bytes of one id written to LDS at p (no bounds: the tile's staged
// output fits the stage).
template <int KIND>
__device__ __forceinline__ void stage_token(const DecodeArgs &a, int32_t id, uint8_t *p) {
    if (is_silent(id)) return;
    if (KIND == DNATOK_KMER) {
        // digit j (most significant first) is the letter at p[j]; unknown
        // ids decode to k letters N (0x4E in every byte)
        const bool known = id >= 5 && id < a.vocab;
        const uint32_t v = (uint32_t)(id - 5);
#pragma unroll 1
        for (int j = 0; j < a.k; ++j)
            p[j] = known ? base_letter(v >> (2 * (a.k - 1 - j))) : (uint8_t)'N';
        return;
    }
    if (KIND == DNATOK_BPE && id >= 10 && id < a.vocab) {
        const int64_t L = a.tok_len[id], o = a.tok_off[id];
#pragma unroll 1
        for (int64_t j = 0; j < L; ++j) p[j] = a.tok_chars[o + j];
        return;
    }
    p[0] = single_letter(id);
}

// A thread's k-mer tokens to the stage from p on, k fixed at compile time
// (digit shifts and store offsets become constants: the runtime-k loop cost
// a dozen instructions per byte and, with every workgroup resident at once,
// made the staging VALU-bound).
template <int K>
__device__ __forceinline__ void stage_kmers(const DecodeArgs &a, const int32_t (&idv)[TPT], uint8_t *p) {
#pragma unroll
    for (int j = 0; j < TPT; ++j) {
        const int32_t id = idv[j];
        if (is_silent(id)) continue;
        const bool known = id >= 5 && id < a.vocab;
        const uint32_t v = (uint32_t)(id - 5);
#pragma unroll
        for (int q = 0; q < K; ++q) p[q] = known ? base_letter(v >> (2 * (K - 1 - q))) : (uint8_t)'N';
        p += K;
    }
}

// The ids of tile t this thread holds (TPT consecutive positions; ids
// outside the rows read as PAD, which decodes to nothing). Every load is
// unconditional, so a thread's loads go out together: a tile inside the rows
// reads its TPT ids as 16-byte vectors, other tiles read clamped positions
// and select.
template <int KIND>
__device__ __forceinline__ int64_t load_tile_ids(const DecodeArgs &a, int64_t t, int64_t first, int64_t last,
                                                 int32_t (&idv)[TPT]) {
    const int64_t p0 = t * TT + (int64_t)threadIdx.x * TPT;
    const bool inside = t * TT >= first && (t + 1) * TT <= last && (t + 1) * TT <= a.n_ids &&
                        (reinterpret_cast<uintptr_t>(a.ids) & 15) == 0;  // uniform over the block
    if (inside) {
        const int4 *q = reinterpret_cast<const int4 *>(a.ids + p0);
#pragma unroll
        for (int j = 0; j < TPT; j += 4) {
            const int4 v = q[j / 4];
            idv[j] = v.x;
            idv[j + 1] = v.y;
            idv[j + 2] = v.z;
            idv[j + 3] = v.w;
        }
    } else if (a.n_ids > 0) {
        int32_t v[TPT];
#pragma unroll
        for (int j = 0; j < TPT; ++j) {
            const int64_t p = p0 + j;
            const bool live = p >= first && p < last && p < a.n_ids && p >= 0;
            v[j] = a.ids[live ? p : 0];
        }
#pragma unroll
        for (int j = 0; j < TPT; ++j) {
            const int64_t p = p0 + j;
            const bool live = p >= first && p < last && p < a.n_ids && p >= 0;
            idv[j] = live ? v[j] : DNATOK_ID_PAD;
        }
    } else {
#pragma unroll
        for (int j = 0; j < TPT; ++j) idv[j] = DNATOK_ID_PAD;
    }
    int32_t mine = 0;  // a thread's 16 tokens of at most 2^20 bases each: 32 bits
#pragma unroll
    for (int j = 0; j < TPT; ++j) mine += width_of<KIND>(a, idv[j]);
    return mine;
}

// 1. The row pass: the first row of every tile, the offsets check, and the
// tile status words cleared for the write pass. Row i is the first row at or
// after position t * TT exactly for the tiles t with
// floor(off[i-1] / TT) < t <= floor(off[i] / TT) (row n stands for the end:
// every tile past the last row start). Bad offsets only raise the flag; the
// tile range is clamped, and the write pass clamps what it reads.
__global__ __launch_bounds__(NT) void k_decode_rows(DecodeArgs a) {
    uint32_t err = 0;
    const int64_t G = (int64_t)gridDim.x * NT;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i <= a.n; i += G) {
        const int64_t prev = (i == 0) ? -1 : a.offs[i - 1];
        const int64_t cur = (i == a.n) ? -1 : a.offs[i];
        if (i < a.n && (cur < 0 || (i + 1 <= a.n && a.offs[i + 1] < cur) || a.offs[i + 1] > a.n_ids))
            err |= DNATOK_DERR_OFFSETS;
        int64_t lo = (i == 0) ? 0 : (prev < 0 ? 0 : prev / a.tt + 1);
        int64_t hi = (i == a.n) ? a.ntiles : (cur < 0 ? -1 : cur / a.tt);
        if (hi > a.ntiles) hi = a.ntiles;
        for (int64_t t = lo; t <= hi; ++t) a.first_row[t] = i;
    }
    for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < a.ntiles; t += G) a.status[t] = 0;
    if (err) dev::raise_error(a.err_hdr, err);
}

// The staged output of a tile (agg bytes from stage byte 0) to out + base:
// output byte base + b is stage byte b, for b below the capacity (past it:
// the flag); the output's 16-byte units from out + base - ph on, each read
// from the stage as 5 dwords realigned by ph.
__device__ __forceinline__ void store_stage(const DecodeArgs &a, const uint8_t *s_out, int64_t base, int64_t agg,
                                            uint32_t &err) {
    const int tid = threadIdx.x;
    const int64_t room = a.cap - base;
    const int64_t lim = room <= 0 ? 0 : (room < agg ? room : agg);
    if (lim < agg) err |= DNATOK_DERR_CAPACITY;
    const int64_t ph = (int64_t)((reinterpret_cast<uintptr_t>(a.out) + (uintptr_t)base) & 15);
    uint8_t *ob = a.out + base - ph;
    const uint32_t *s32 = reinterpret_cast<const uint32_t *>(s_out);
    const int64_t nu = lim > 0 ? (ph + lim + 15) / 16 : 0;
    for (int64_t u = tid; u < nu; u += NT) {
        const int64_t lo = 16 * u - ph, hi = lo + 16;  // the unit's stage bytes
        if (lo >= 0 && hi <= lim) {
            const uint32_t w0 = (uint32_t)lo >> 2, r = (uint32_t)lo & 3;
            uint32_t w[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) w[q] = s32[w0 + q];
            uint4 o;
            o.x = __builtin_amdgcn_alignbyte(w[1], w[0], r);
            o.y = __builtin_amdgcn_alignbyte(w[2], w[1], r);
            o.z = __builtin_amdgcn_alignbyte(w[3], w[2], r);
            o.w = __builtin_amdgcn_alignbyte(w[4], w[3], r);
            *reinterpret_cast<uint4 *>(ob + 16 * u) = o;
        } else {
            for (int64_t b = (lo > 0 ? lo : 0); b < hi && b < lim; ++b) ob[ph + b] = s_out[b];
        }
    }
}

// 2. One workgroup per tile (tile = workgroup index): the tile's ids are
// read once; their byte total is published for later tiles before the
// look-back, which wave 0 runs while the other waves stage the tile's bytes
// in LDS. Once the output position is known, the block writes the output's
// 16-byte units (each read from the stage realigned to the output's phase;
// partial first and last units byte by byte), up to the capacity (past it:
// the flag); a tile whose output exceeds the stage writes its tokens
// directly. Rows starting in the tile get their output offsets; the last
// tile writes the total.
template <int KIND>
__global__ __launch_bounds__(NT) void k_decode_write(DecodeArgs a) {
    extern __shared__ __align__(16) uint8_t s_out[];
    __shared__ int64_t s_tpre[NT + 1];  // in-tile bytes before each thread's first position (and the total)
    __shared__ int64_t s_tmp[NT / dev::kWave + 1];
    __shared__ int64_t s_ia, s_ib, s_base;
    const int tid = threadIdx.x;
    const int64_t t = blockIdx.x;
    const int64_t P0 = t * TT;
    // the tile's rows go out with its ids (neither depends on the other)
    int64_t ia = 0, ib = 0;
    if (tid == 0) {
        ia = a.first_row[t];
        ib = (t == a.ntiles - 1) ? a.n : a.first_row[t + 1];
    }
    const int64_t first = (a.n > 0) ? a.offs[0] : 0;
    const int64_t last = (a.n > 0) ? a.offs[a.n] : 0;
    int32_t idv[TPT];
    const int64_t mine = load_tile_ids<KIND>(a, t, first, last, idv);
    int64_t agg;
    const int64_t pre = dev::block_excl_scan<NT>(mine, s_tmp, &agg);
    if (tid < dev::kWave) {
        if (tid == 0) dev::publish_aggregate(a.status, t, agg);
        const int64_t excl = dev::wave_lookback(a.status, t, agg, a.err_hdr);
        if (tid == 0) {
            // rows starting in the tile (clamped: bad offsets leave the
            // table unchecked, and they raise the flag in the row pass)
            ia = ia < 0 ? 0 : (ia > a.n ? a.n : ia);
            ib = ib < ia ? ia : (ib > a.n ? a.n : ib);
            s_ia = ia;
            s_ib = ib;
            s_base = excl;
        }
    }
    s_tpre[tid] = pre;
    if (tid == NT - 1) s_tpre[NT] = pre + mine;
    // The bytes go to LDS from stage offset 0 while wave 0 still waits on
    // the look-back (their output position matters only to the stores).
    const bool staged = agg <= a.stage;
    if (staged) {
        // in-tile positions fit 32 bits (the stage is at most 32 KiB)
        uint32_t pos = (uint32_t)pre;
        if (KIND == DNATOK_KMER && a.k <= 8) {
            uint8_t *p = s_out + pos;
            switch (a.k) {
            case 1: stage_kmers<1>(a, idv, p); break;
            case 2: stage_kmers<2>(a, idv, p); break;
            case 3: stage_kmers<3>(a, idv, p); break;
            case 4: stage_kmers<4>(a, idv, p); break;
            case 5: stage_kmers<5>(a, idv, p); break;
            case 6: stage_kmers<6>(a, idv, p); break;
            case 7: stage_kmers<7>(a, idv, p); break;
            default: stage_kmers<8>(a, idv, p); break;
            }
        } else {
#pragma unroll
            for (int j = 0; j < TPT; ++j) {
                stage_token<KIND>(a, idv[j], s_out + pos);
                pos += (uint32_t)width_of<KIND>(a, idv[j]);
            }
        }
    }
    __syncthreads();
    const int64_t base = s_base;
    uint32_t err = 0;
    if (staged) {
        store_stage(a, s_out, base, agg, err);
    } else {
        // rare (output over the stage): the ids again, one at a time from
        // the cache, written straight to the output
        int64_t pos = base + pre;
        const int64_t p0 = t * TT + (int64_t)tid * TPT;
#pragma unroll 1
        for (int j = 0; j < TPT; ++j) {
            const int64_t q = p0 + j;
            const bool live = q >= first && q < last && q < a.n_ids;
            const int32_t id = live ? a.ids[q] : DNATOK_ID_PAD;
            write_token<KIND>(a, id, pos, err);
            pos += width_of<KIND>(a, id);
        }
    }
    // rows starting in the tile: the bytes before their first position are
    // the owning thread's prefix plus its ids before that position (read
    // again from the cache; a tile holds a few row starts)
    for (int64_t i = s_ia + tid; i < s_ib; i += NT) {
        int64_t rel = a.offs[i] - P0;
        rel = rel < 0 ? 0 : (rel > TT ? TT : rel);
        const int th = (int)(rel / TPT);
        int64_t sum = s_tpre[th];
        for (int64_t q = P0 + (int64_t)th * TPT; q < P0 + rel; ++q) {
            const bool live = q >= first && q < last && q < a.n_ids;
            sum += width_of<KIND>(a, live ? a.ids[q] : DNATOK_ID_PAD);
        }
        a.out_offs[i] = base + sum;
    }
    if (t == a.ntiles - 1 && tid == 0) a.out_offs[a.n] = base + agg;
    if (err) dev::raise_error(a.err_hdr, err);
}


// 2'. The same for single-nucleotide and k-mer vocabularies up to 8 bases
// (every token K bytes or none, a tile's output always staged), with the
// ids strided: thread i holds the tile's ids i, i + NT, ..., so a wave's
// lanes hold 64 consecutive ids. Loads coalesce per instruction, and a
// staged byte store's lanes land on consecutive dwords; with each thread
// holding 16 consecutive ids, one store's lanes were 96 bytes apart, on a
// few LDS banks, and the staging ran bank-conflict bound beside the
// look-back. Positions: a wave's ballot of the non-silent ids of slice j
// gives each lane its count below it; one scan over the 64 (slice, wave)
// counts in id order gives the rest. The ballots also give the row starts.
template <int KIND, int K, int TPS>
__global__ __launch_bounds__(NT) void k_decode_strided(DecodeArgs a) {
    constexpr int NW = NT / dev::kWave;
    constexpr int TPT = TPS, TT = NT * TPS;  // this kernel's ids per thread and per tile
    constexpr int NS = TPT * NW;             // (slice, wave) entries, a multiple of the wave
    extern __shared__ __align__(16) uint8_t s_out[];
    __shared__ uint32_t s_cnt[NS + 1];  // per (slice, wave): non-silent ids, then ids before; [NS]: total
    __shared__ uint64_t s_msk[NS];      // per (slice, wave): which lanes hold a non-silent id
    __shared__ int64_t s_ia, s_ib, s_base;
    const int tid = threadIdx.x, lane = tid & (dev::kWave - 1), w = tid / dev::kWave;
    const int64_t t = blockIdx.x;
    const int64_t P0 = t * TT;
    if (tid == 0) {
        int64_t ia = a.first_row[t];
        int64_t ib = (t == a.ntiles - 1) ? a.n : a.first_row[t + 1];
        // rows starting in the tile (clamped: bad offsets raise the flag in the row pass)
        ia = ia < 0 ? 0 : (ia > a.n ? a.n : ia);
        ib = ib < ia ? ia : (ib > a.n ? a.n : ib);
        s_ia = ia;
        s_ib = ib;
    }
    const int64_t first = (a.n > 0) ? a.offs[0] : 0;
    const int64_t last = (a.n > 0) ? a.offs[a.n] : 0;
    // ids outside the rows read as PAD (no output); loads are unconditional
    // (clamped) so they go out together
    int32_t idv[TPT];
#pragma unroll
    for (int j = 0; j < TPT; ++j) {
        const int64_t p = P0 + (int64_t)j * NT + tid;
        const bool live = p >= first && p < last && p < a.n_ids;
        const int32_t v = a.n_ids > 0 ? a.ids[live ? p : 0] : 0;
        idv[j] = live ? v : DNATOK_ID_PAD;
    }
    uint32_t below[TPT];  // non-silent ids of this slice and wave below this lane
#pragma unroll
    for (int j = 0; j < TPT; ++j) {
        const uint64_t m = __ballot(!is_silent(idv[j]));
        below[j] = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (lane == 0) {
            s_cnt[j * NW + w] = (uint32_t)__popcll(m);
            s_msk[j * NW + w] = m;
        }
    }
    __syncthreads();
    if (tid < dev::kWave) {  // ids before each (slice, wave), in id order; a lane takes NS / 64 in a row
        constexpr int PER = NS / dev::kWave;
        uint32_t v[PER], sum = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            v[q] = s_cnt[tid * PER + q];
            sum += v[q];
        }
        const uint32_t inc = dev::wave_incl_sum_u32(sum);
        uint32_t run = inc - sum;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            s_cnt[tid * PER + q] = run;
            run += v[q];
        }
        if (tid == dev::kWave - 1) s_cnt[NS] = inc;
    }
    __syncthreads();
    const int64_t agg = (int64_t)K * s_cnt[NS];
    if (tid < dev::kWave) {
        if (tid == 0) dev::publish_aggregate(a.status, t, agg);
        const int64_t excl = dev::wave_lookback(a.status, t, agg, a.err_hdr);
        if (tid == 0) s_base = excl;
    }
    // the bytes go to LDS while wave 0 still waits on the look-back
#pragma unroll
    for (int j = 0; j < TPT; ++j) {
        const int32_t id = idv[j];
        if (is_silent(id)) continue;
        uint8_t *p = s_out + (uint32_t)K * (s_cnt[j * NW + w] + below[j]);
        if (KIND == DNATOK_SINGLE) {
            p[0] = single_letter(id);
        } else {
            const bool known = id >= 5 && id < a.vocab;
            const uint32_t v = (uint32_t)(id - 5);
#pragma unroll
            for (int q = 0; q < K; ++q) p[q] = known ? base_letter(v >> (2 * (K - 1 - q))) : (uint8_t)'N';
        }
    }
    __syncthreads();
    const int64_t base = s_base;
    uint32_t err = 0;
    store_stage(a, s_out, base, agg, err);
    // rows starting in the tile: K bytes per non-silent id before their first position
    for (int64_t i = s_ia + tid; i < s_ib; i += NT) {
        int64_t rel = a.offs[i] - P0;
        rel = rel < 0 ? 0 : (rel > TT ? TT : rel);
        uint32_t c = s_cnt[NS];
        if (rel < TT) {
            const int js = (int)(rel / NT), ws = (int)((rel % NT) / dev::kWave), l = (int)(rel % dev::kWave);
            c = s_cnt[js * NW + ws] + (uint32_t)__popcll(s_msk[js * NW + ws] & ((1ull << l) - 1ull));
        }
        a.out_offs[i] = base + (int64_t)K * c;
    }
    if (t == a.ntiles - 1 && tid == 0) a.out_offs[a.n] = base + agg;
    if (err) dev::raise_error(a.err_hdr, err);
}

}  // namespace

int launch_decode(const dnatok_vocab *v, const int32_t *d_ids, int64_t n_ids, const int64_t *d_offsets, int32_t n,
                  uint8_t *d_out, int64_t out_capacity, int64_t *d_out_offsets, hipStream_t stream) {
    DecodeArgs a;
    a.ids = d_ids;
    a.n_ids = n_ids;
    a.offs = d_offsets;
    a.n = n;
    a.out = d_out;
    a.cap = out_capacity;
    a.out_offs = d_out_offsets;
    a.kind = v->kind;
    a.k = v->k;
    a.vocab = v->vocab_size;
    a.tok_len = v->bpe.d_tok_len;
    a.tok_off = v->bpe.d_tok_off;
    a.tok_chars = v->bpe.d_tok_chars;
    // single-nucleotide ids go 32 per thread (8,192 per tile): half the tiles'
    // fixed latency for a stage of 8 KiB (73 -> 58 us for 33.6M ids)
    a.tt = v->kind == DNATOK_SINGLE ? (int64_t)TT_SINGLE : (int64_t)TT;
    a.ntiles = n_ids / a.tt + 1;
    if (a.ntiles >= (1ll << 31)) return set_error(DNATOK_EINVAL, "too many ids for one decode");
    // the stage holds a tile's output at the vocabulary's widest token
    const int64_t wmax = v->kind == DNATOK_KMER ? v->k : (v->kind == DNATOK_BPE ? v->max_token_bytes : 1);
    a.stage = (int32_t)std::min<int64_t>(a.tt * std::max<int64_t>(wmax, 1), kMaxStage);
    Workspace *ws = nullptr;
    int rc = get_workspace(stream, 1, &ws);
    if (rc) return rc;
    rc = ensure_scratch(ws, 16 * (a.ntiles + 1));
    if (rc) return rc;
    a.status = reinterpret_cast<uint64_t *>(ws->d_scratch);
    a.first_row = reinterpret_cast<int64_t *>(a.status + (a.ntiles + 1));
    a.err_hdr = ws->d_hdr;
    const int64_t rows_grid = std::min<int64_t>(((int64_t)n + 1 + NT - 1) / NT + 1, 4ll * device_cu_count());
    hipLaunchKernelGGL(k_decode_rows, dim3((unsigned)std::max<int64_t>(rows_grid, 1)), dim3(NT), 0, stream, a);
    DNATOK_HIP(hipGetLastError());
    const dim3 grid((unsigned)a.ntiles), block(NT);
    const size_t dyn = (size_t)a.stage + 16;  // a unit's realigning reads go up to 3 bytes past the data
    if (v->kind == DNATOK_SINGLE) {  // its stage (a.tt bytes) always holds the tile
        hipLaunchKernelGGL((k_decode_strided<DNATOK_SINGLE, 1, TPT_SINGLE>), grid, block, dyn, stream, a);
    } else if (v->kind == DNATOK_KMER && v->k <= 8 && a.stage >= TT * v->k) {
        switch (v->k) {
        case 1: hipLaunchKernelGGL((k_decode_strided<DNATOK_KMER, 1, TPT>), grid, block, dyn, stream, a); break;
        case 2: hipLaunchKernelGGL((k_decode_strided<DNATOK_KMER, 2, TPT>), grid, block, dyn, stream, a); break;
        case 3: hipLaunchKernelGGL((k_decode_strided<DNATOK_KMER, 3, TPT>), grid, block, dyn, stream, a); break;
        case 4: hipLaunchKernelGGL((k_decode_strided<DNATOK_KMER, 4, TPT>), grid, block, dyn, stream, a); break;
        case 5: hipLaunchKernelGGL((k_decode_strided<DNATOK_KMER, 5, TPT>), grid, block, dyn, stream, a); break;
        case 6: hipLaunchKernelGGL((k_decode_strided<DNATOK_KMER, 6, TPT>), grid, block, dyn, stream, a); break;
        case 7: hipLaunchKernelGGL((k_decode_strided<DNATOK_KMER, 7, TPT>), grid, block, dyn, stream, a); break;
        default: hipLaunchKernelGGL((k_decode_strided<DNATOK_KMER, 8, TPT>), grid, block, dyn, stream, a); break;
        }
    } else if (v->kind == DNATOK_KMER)
        hipLaunchKernelGGL(k_decode_write<DNATOK_KMER>, grid, block, dyn, stream, a);
    else
        hipLaunchKernelGGL(k_decode_write<DNATOK_BPE>, grid, block, dyn, stream, a);
    DNATOK_HIP(hipGetLastError());
    return DNATOK_OK;
}

}  // namespace dnatok
