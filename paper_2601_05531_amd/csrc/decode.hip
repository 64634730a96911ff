// Decode: ids -> uppercase bases (the inverse table the paper lists as
// future work, Discussion, "Decode Operations": the same LUT principle run
// backwards). Not on the hot path.
//
// Tiles of TT token positions, each tile's output bytes contiguous. Three
// launches: per-tile byte totals, their scan (one workgroup), and the write,
// where each tile stages its bytes in LDS and writes them with 16-byte
// stores. No tile waits on another and no ticket counter is involved (one
// device-wide counter serializes at about 12 ns per ticket, which at
// tens of thousands of tiles outweighs the decode itself).
#include "common.hpp"
#include "device.hpp"

namespace dnatok {

namespace {

constexpr int NT = 256;
constexpr int TPT = 8;  // tokens per thread
constexpr int TT = NT * TPT;
constexpr int kStage = 16384;  // bytes of one tile's output staged in LDS (2,048 k-mers of k <= 8)

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
    int64_t *tile_pre;   // per-tile output bytes, then their exclusive scan (ntiles + 1)
    int64_t *first_row;  // first row starting at or after each tile's first position (ntiles + 1)
    uint32_t *err_hdr;
};

__device__ __forceinline__ bool is_silent(int32_t id) {
    return id == DNATOK_ID_PAD || id == DNATOK_ID_CLS || id == DNATOK_ID_SEP || id == DNATOK_ID_MASK;
}

__device__ __forceinline__ int64_t width_of(const DecodeArgs &a, int32_t id) {
    if (is_silent(id)) return 0;
    if (a.kind == DNATOK_KMER) return a.k;
    if (a.kind == DNATOK_BPE && id >= 10 && id < a.vocab) return a.tok_len[id];
    return 1;
}

__device__ __forceinline__ void write_token(const DecodeArgs &a, int32_t id, int64_t pos, uint32_t &err) {
    if (is_silent(id)) return;
    const uint8_t base4[4] = {'A', 'C', 'G', 'T'};
    if (a.kind == DNATOK_KMER) {
        const bool known = id >= 5 && id < a.vocab;
        uint32_t v = known ? (uint32_t)(id - 5) : 0u;
        for (int j = a.k - 1; j >= 0; --j) {
            int64_t p = pos + j;
            if (p < a.cap) a.out[p] = known ? base4[v & 3] : (uint8_t)'N';
            else err |= DNATOK_DERR_CAPACITY;
            v >>= 2;
        }
        return;
    }
    if (a.kind == DNATOK_BPE && id >= 10 && id < a.vocab) {
        const int64_t L = a.tok_len[id], o = a.tok_off[id];
        for (int64_t j = 0; j < L; ++j) {
            if (pos + j < a.cap) a.out[pos + j] = a.tok_chars[o + j];
            else err |= DNATOK_DERR_CAPACITY;
        }
        return;
    }
    uint8_t c = (id >= 5 && id <= 8) ? base4[id - 5] : (uint8_t)'N';
    if (pos < a.cap) a.out[pos] = c;
    else err |= DNATOK_DERR_CAPACITY;
}

// Slot of tile position q (thread q / TPT, its j = q % TPT) in the prefix
// table: j * NT + thread, so the TPT writes of a wave each hit consecutive
// slots (thread-major order would put every lane of a write on two banks).
__device__ __forceinline__ int32_t pre_slot(int32_t q) { return (q % TPT) * NT + q / TPT; }

// The bytes of one id written to LDS at p (no bounds: the tile's staged
// output fits the stage).
__device__ __forceinline__ void stage_token(const DecodeArgs &a, int32_t id, uint8_t *p) {
    if (is_silent(id)) return;
    if (a.kind == DNATOK_KMER) {
        const bool known = id >= 5 && id < a.vocab;
        uint32_t v = known ? (uint32_t)(id - 5) : 0u;
        for (int j = a.k - 1; j >= 0; --j) {
            p[j] = known ? (uint8_t)"ACGT"[v & 3] : (uint8_t)'N';
            v >>= 2;
        }
        return;
    }
    if (a.kind == DNATOK_BPE && id >= 10 && id < a.vocab) {
        const int64_t L = a.tok_len[id], o = a.tok_off[id];
        for (int64_t j = 0; j < L; ++j) p[j] = a.tok_chars[o + j];
        return;
    }
    p[0] = (id >= 5 && id <= 8) ? (uint8_t)"ACGT"[id - 5] : (uint8_t)'N';
}

// The ids of tile t this thread holds (TPT consecutive positions; ids
// outside the rows read as PAD, which decodes to nothing). Every load is
// unconditional, so a thread's loads go out together: a tile inside the rows
// reads its TPT ids as 16-byte vectors, other tiles read clamped positions
// and select.
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
    int64_t mine = 0;
#pragma unroll
    for (int j = 0; j < TPT; ++j) mine += width_of(a, idv[j]);
    return mine;
}

// 1. Output bytes of every tile, CT tiles per pass so each thread has
// CT * TPT ids in flight; the first row of every tile; the offsets check.
// Row i is the first row at or after position t * TT exactly for the tiles t
// with floor(off[i-1] / TT) < t <= floor(off[i] / TT) (row n stands for the
// end: every tile past the last row start). Bad offsets only raise the flag;
// the tile range is clamped, and the write pass clamps what it reads.
__global__ __launch_bounds__(NT) void k_decode_count(DecodeArgs a) {
    constexpr int CT = 4;
    __shared__ int64_t s_part[NT / dev::kWave][CT];
    const int64_t first = (a.n > 0) ? a.offs[0] : 0;
    const int64_t last = (a.n > 0) ? a.offs[a.n] : 0;
    const int w = threadIdx.x / dev::kWave, lane = threadIdx.x & (dev::kWave - 1);
    uint32_t err = 0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i <= a.n; i += (int64_t)gridDim.x * NT) {
        const int64_t prev = (i == 0) ? -1 : a.offs[i - 1];
        const int64_t cur = (i == a.n) ? -1 : a.offs[i];
        if (i < a.n && (cur < 0 || (i + 1 <= a.n && a.offs[i + 1] < cur) || a.offs[i + 1] > a.n_ids))
            err |= DNATOK_DERR_OFFSETS;
        int64_t lo = (i == 0) ? 0 : (prev < 0 ? 0 : prev / TT + 1);
        int64_t hi = (i == a.n) ? a.ntiles : (cur < 0 ? -1 : cur / TT);
        if (hi > a.ntiles) hi = a.ntiles;
        for (int64_t t = lo; t <= hi; ++t) a.first_row[t] = i;
    }
    for (int64_t t0 = (int64_t)blockIdx.x * CT; t0 < a.ntiles; t0 += (int64_t)gridDim.x * CT) {
        int32_t idv[CT][TPT];
        int64_t part[CT];
        const bool inside = t0 * TT >= first && (t0 + CT) * TT <= last && (t0 + CT) * TT <= a.n_ids &&
                            (reinterpret_cast<uintptr_t>(a.ids) & 15) == 0;  // uniform over the block
        if (inside) {
            // all CT tiles inside the rows: every load of the pass goes out at once
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const int4 *q = reinterpret_cast<const int4 *>(a.ids + (t0 + c) * TT + (int64_t)threadIdx.x * TPT);
#pragma unroll
                for (int j = 0; j < TPT; j += 4) {
                    const int4 v = q[j / 4];
                    idv[c][j] = v.x;
                    idv[c][j + 1] = v.y;
                    idv[c][j + 2] = v.z;
                    idv[c][j + 3] = v.w;
                }
            }
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                part[c] = 0;
#pragma unroll
                for (int j = 0; j < TPT; ++j) part[c] += width_of(a, idv[c][j]);
            }
        } else {
#pragma unroll
            for (int c = 0; c < CT; ++c) part[c] = load_tile_ids(a, t0 + c, first, last, idv[c]);
        }
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int64_t v = dev::wave_sum(part[c]);
            if (lane == 0) s_part[w][c] = v;
        }
        __syncthreads();
        if (threadIdx.x < CT && t0 + threadIdx.x < a.ntiles) {
            int64_t sum = 0;
            for (int q = 0; q < NT / dev::kWave; ++q) sum += s_part[q][threadIdx.x];
            a.tile_pre[t0 + threadIdx.x] = sum;
        }
        __syncthreads();
    }
    if (err) dev::raise_error(a.err_hdr, err);
}

// 2. Exclusive scan of the tile totals in place (one workgroup); the total
// goes to tile_pre[ntiles] and out_offs[n].
__global__ __launch_bounds__(NT) void k_decode_scan(DecodeArgs a) {
    __shared__ int64_t s_tmp[NT / dev::kWave + 1];
    constexpr int PER = 16;
    int64_t run = 0;
    for (int64_t c0 = 0; c0 < a.ntiles; c0 += (int64_t)NT * PER) {
        const int64_t i0 = c0 + (int64_t)threadIdx.x * PER;
        int64_t v[PER];
        int64_t mine = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            // unconditional load of a clamped entry (ntiles >= 1), so the
            // thread's loads go out together
            const int64_t x = a.tile_pre[i0 + j < a.ntiles ? i0 + j : a.ntiles - 1];
            v[j] = (i0 + j < a.ntiles) ? x : 0;
            mine += v[j];
        }
        int64_t tot;
        int64_t pre = run + dev::block_excl_scan<NT>(mine, s_tmp, &tot);
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            if (i0 + j < a.ntiles) a.tile_pre[i0 + j] = pre;
            pre += v[j];
        }
        run += tot;
    }
    if (threadIdx.x == 0) {
        a.tile_pre[a.ntiles] = run;
        a.out_offs[a.n] = run;
    }
}

// 3. Each tile's bytes, staged in LDS at their 16-byte phase in the output
// and written with 16-byte stores (partial first and last units byte by
// byte); a tile whose output exceeds the stage, or that would cross the
// capacity, writes its tokens directly. Rows starting in the tile get their
// output offsets.
__global__ __launch_bounds__(NT) void k_decode_write(DecodeArgs a) {
    __shared__ __align__(16) uint8_t s_out[kStage + 16];
    __shared__ int32_t s_pre[TT + 1];  // bytes before each tile position (in-tile, so 32-bit), position-major
    __shared__ int64_t s_tmp[NT / dev::kWave + 1];
    __shared__ int64_t s_ia, s_ib;
    const int tid = threadIdx.x;
    const int64_t first = (a.n > 0) ? a.offs[0] : 0;
    const int64_t last = (a.n > 0) ? a.offs[a.n] : 0;
    uint32_t err = 0;
    for (int64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const int64_t P0 = t * TT, P1 = P0 + TT;
        int32_t idv[TPT];
        const int64_t mine = load_tile_ids(a, t, first, last, idv);
        int64_t agg;
        const int64_t pre = dev::block_excl_scan<NT>(mine, s_tmp, &agg);
        {
            int64_t run = pre;
#pragma unroll
            for (int j = 0; j < TPT; ++j) {
                s_pre[pre_slot(tid * TPT + j)] = (int32_t)run;  // lanes write consecutive slots: no bank conflicts
                run += width_of(a, idv[j]);
            }
            if (tid == NT - 1) s_pre[TT] = (int32_t)run;
        }
        if (tid == 0) {
            // rows starting in the tile (clamped: bad offsets leave the
            // table unchecked, and they raise the flag in the count pass)
            int64_t ia = a.first_row[t], ib = (t == a.ntiles - 1) ? a.n : a.first_row[t + 1];
            ia = ia < 0 ? 0 : (ia > a.n ? a.n : ia);
            ib = ib < ia ? ia : (ib > a.n ? a.n : ib);
            s_ia = ia;
            s_ib = ib;
        }
        const int64_t base = a.tile_pre[t];
        const int64_t ph = (int64_t)((reinterpret_cast<uintptr_t>(a.out) + (uintptr_t)base) & 15);
        const bool staged = agg <= kStage && base + agg <= a.cap;
        if (staged) {
            int64_t pos = pre;
#pragma unroll
            for (int j = 0; j < TPT; ++j) {
                stage_token(a, idv[j], s_out + ph + pos);
                pos += width_of(a, idv[j]);
            }
        } else {
            int64_t pos = base + pre;
#pragma unroll
            for (int j = 0; j < TPT; ++j) {
                write_token(a, idv[j], pos, err);
                pos += width_of(a, idv[j]);
            }
        }
        __syncthreads();
        if (staged && agg > 0) {
            // s_out[ph + i] is output byte base + i; unit u covers stage bytes
            // [16u, 16u + 16), i.e. output base - ph + 16u, 16-byte aligned
            uint8_t *ob = a.out + base - ph;
            const int64_t nu = (ph + agg + 15) / 16;
            for (int64_t u = tid; u < nu; u += NT) {
                const int64_t lo = 16 * u, hi = lo + 16;
                if (lo >= ph && hi <= ph + agg) {
                    *reinterpret_cast<uint4 *>(ob + lo) = *reinterpret_cast<const uint4 *>(s_out + lo);
                } else {
                    for (int64_t b = (lo > ph ? lo : ph); b < hi && b < ph + agg; ++b) ob[b] = s_out[b];
                }
            }
        }
        for (int64_t i = s_ia + tid; i < s_ib; i += NT) {
            int64_t rel = a.offs[i] - P0;
            rel = rel < 0 ? 0 : (rel > TT ? TT : rel);
            a.out_offs[i] = base + s_pre[rel == TT ? TT : pre_slot((int32_t)rel)];
        }
        __syncthreads();
    }
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
    a.ntiles = n_ids / TT + 1;
    Workspace *ws = nullptr;
    int rc = get_workspace(stream, 1, &ws);
    if (rc) return rc;
    rc = ensure_scratch(ws, 16 * (a.ntiles + 1));
    if (rc) return rc;
    a.tile_pre = reinterpret_cast<int64_t *>(ws->d_scratch);
    a.first_row = a.tile_pre + (a.ntiles + 1);
    a.err_hdr = ws->d_hdr;
    int per_cu = 0;
    DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_decode_write, NT, 0));
    if (per_cu < 1) per_cu = 1;
    int64_t grid = 4 * (int64_t)device_cu_count() * per_cu;
    if (grid > a.ntiles) grid = a.ntiles;
    hipLaunchKernelGGL(k_decode_count, dim3((unsigned)grid), dim3(NT), 0, stream, a);
    DNATOK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_decode_scan, dim3(1), dim3(NT), 0, stream, a);
    DNATOK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_decode_write, dim3((unsigned)grid), dim3(NT), 0, stream, a);
    DNATOK_HIP(hipGetLastError());
    return DNATOK_OK;
}

}  // namespace dnatok
