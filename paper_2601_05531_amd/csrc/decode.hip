// Decode: ids -> uppercase bases (the inverse table the paper lists as
// future work, Discussion, "Decode Operations": the same LUT principle run
// backwards). Not on the hot path.
//
// One launch, same structure as encode: tiles of TT token positions, each
// tile's output bytes are contiguous, a one-pass look-back turns per-tile
// byte counts into output positions.
#include "common.hpp"
#include "device.hpp"

namespace dnatok {

namespace {

constexpr int NT = 256;
constexpr int TPT = 8;  // tokens per thread
constexpr int TT = NT * TPT;

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
    dev::TileQueue q;
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

__global__ __launch_bounds__(NT) void k_decode(DecodeArgs a) {
    __shared__ int64_t s_pre[TT + 1];
    __shared__ int64_t s_tmp[NT / dev::kWave + 1];
    __shared__ int64_t s_ticket, s_ia, s_ib, s_excl;
    __shared__ uint32_t s_err;
    const int tid = threadIdx.x;
    const uint32_t parity = dev::ld_relaxed32(a.q.hdr + 2);
    uint64_t *st = parity ? a.q.status1 : a.q.status0;
    uint64_t *st_other = parity ? a.q.status0 : a.q.status1;
    const int64_t first = (a.n > 0) ? a.offs[0] : 0;
    const int64_t last = (a.n > 0) ? a.offs[a.n] : 0;

    for (;;) {
        if (tid == 0) {
            s_ticket = (int64_t)atomicAdd(a.q.hdr + 0, 1u);
            s_err = 0;
        }
        __syncthreads();
        const int64_t t = s_ticket;
        if (t >= a.ntiles) break;
        uint32_t err = 0;
        for (int64_t j = t + (int64_t)tid * a.ntiles; j < a.q.clear_n; j += (int64_t)NT * a.ntiles) st_other[j] = 0;
        for (int64_t i = t + (int64_t)tid * a.ntiles; i < a.n; i += (int64_t)NT * a.ntiles) {
            int64_t o0 = a.offs[i], o1 = a.offs[i + 1];
            if (o0 < 0 || o1 < o0 || o1 > a.n_ids) err |= DNATOK_DERR_OFFSETS;
        }
        const int64_t P0 = t * TT;
        const int64_t P1 = P0 + TT;

        int32_t idv[TPT];
        int64_t mine = 0;
#pragma unroll
        for (int j = 0; j < TPT; ++j) {
            const int64_t p = P0 + (int64_t)tid * TPT + j;
            const bool live = p >= first && p < last && p < a.n_ids && p >= 0;
            idv[j] = live ? a.ids[p] : DNATOK_ID_PAD;
            mine += width_of(a, idv[j]);
        }
        int64_t agg;
        int64_t pre = dev::block_excl_scan<NT>(mine, s_tmp, &agg);
        {
            int64_t run = pre;
#pragma unroll
            for (int j = 0; j < TPT; ++j) {
                s_pre[tid * TPT + j] = run;
                run += width_of(a, idv[j]);
            }
            if (tid == NT - 1) s_pre[TT] = run;
        }
        if (tid == 0) {
            s_excl = dev::lookback(st, t, agg);
            int64_t lo = 0, hi = a.n;  // first row with offs[i] >= P0
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                if (a.offs[mid] >= P0) hi = mid;
                else lo = mid + 1;
            }
            s_ia = lo;
            hi = a.n;
            if (t == a.ntiles - 1) {
                lo = a.n;
            } else {
                while (lo < hi) {
                    int64_t mid = (lo + hi) >> 1;
                    if (a.offs[mid] >= P1) hi = mid;
                    else lo = mid + 1;
                }
            }
            s_ib = lo;
        }
        __syncthreads();
        const int64_t base = s_excl;
        int64_t pos = base + pre;
#pragma unroll
        for (int j = 0; j < TPT; ++j) {
            write_token(a, idv[j], pos, err);
            pos += width_of(a, idv[j]);
        }
        for (int64_t i = s_ia + tid; i < s_ib; i += NT) {
            int64_t rel = a.offs[i] - P0;
            rel = rel < 0 ? 0 : (rel > TT ? TT : rel);
            a.out_offs[i] = base + s_pre[rel];
        }
        if (t == a.ntiles - 1 && tid == 0) a.out_offs[a.n] = base + agg;
        if (err) atomicOr(&s_err, err);
        __syncthreads();
        if (tid == 0 && s_err) dev::raise_error(a.q.hdr, s_err);
    }
    if (tid == 0) dev::finish_block(a.q.hdr);
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
    int rc = get_workspace(stream, a.ntiles, &ws);
    if (rc) return rc;
    a.q.hdr = ws->d_hdr;
    a.q.status0 = ws->d_status;
    a.q.status1 = ws->d_status + ws->cap;
    if (a.ntiles > ws->high_water) ws->high_water = a.ntiles;
    a.q.clear_n = ws->high_water;
    int per_cu = 0;
    DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_decode, NT, 0));
    if (per_cu < 1) per_cu = 1;
    int64_t grid = (int64_t)device_cu_count() * per_cu;
    if (grid > a.ntiles) grid = a.ntiles;
    hipLaunchKernelGGL(k_decode, dim3((unsigned)grid), dim3(NT), 0, stream, a);
    DNATOK_HIP(hipGetLastError());
    return DNATOK_OK;
}

}  // namespace dnatok
