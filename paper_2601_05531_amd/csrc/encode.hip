// Byte -> identifier encode of a ragged batch in one persistent HIP launch.
//
// Paper: Design, "Encoding paths", bytes path (device-resident 256-entry LUT
// applied to staged ASCII) and the bytes branch of the EmbedFromStrings
// algorithm (MapKmer for k-mer vocabularies, left padding to token_len).
//
// Work decomposition (MI355X-first; the paper applies ascii_lut[Bytes] as a
// framework tensor op on an equal-length B x T matrix):
//  * The concatenated input is cut into fixed tiles of B bytes (B a multiple
//    of 16, addressed from the 16-byte-aligned base so every tile load is a
//    full 16-byte vector load). Every output cell is owned by the tile that
//    holds its anchor byte: CLS at the row start, body token j at
//    off + j*k, SEP at the row's last byte, pads at the CLS (left) or SEP
//    (right) anchor. A tile therefore owns one contiguous run of cells per
//    row it touches, and its PACKED output is one contiguous range, so the
//    work per tile is bounded by B whatever the row lengths are.
//  * Output positions need the token count of all earlier tiles: a one-pass
//    decoupled look-back over per-tile counts (tickets hand tiles out in
//    order, so a tile only ever waits on tiles that are already running).
//  * The tile's bytes are staged into LDS once with coalesced 16-byte loads.
//    k-mer tiles are classified on the way in: 2-bit base digits packed
//    most-significant-first (16 bases per word) plus one validity bit per
//    base, so a k-mer id is one 64-bit funnel shift and one mask compare.
//    Single-base tiles keep raw bytes and the 256-entry table sits in LDS.
//  * Stores go out as aligned 16-byte groups of four ids (plus one 4-byte
//    mask word in PADDED layout); ragged group edges fall back to scalar
//    stores.
#include "common.hpp"
#include "device.hpp"

namespace dnatok {

namespace {

constexpr int NT = 256;

struct EncodeArgs {
    const uint8_t *abase;  // input base aligned down to 16 bytes
    int64_t shift;         // d_bytes - abase
    int64_t nbytes;
    const int64_t *offs;
    int32_t n;
    int32_t k;
    int32_t *ids;
    int64_t cap;
    int64_t *out_offs;
    int8_t *mask;
    const int32_t *lut;
    int32_t cls;
    int32_t padded;
    int32_t left;
    int32_t pad_id, cls_id, sep_id;
    int64_t W;
    int64_t base;
    int64_t tileB;
    int64_t ntiles;
    dev::TileQueue q;
};

// Number of body tokens of a row of L bytes.
__device__ __forceinline__ int64_t body_tokens(int64_t L, int32_t k, bool kmer) {
    return kmer ? (L + k - 1) / k : L;
}

struct Row {
    int64_t off, end, nb, len;
};

// Tokens of the row whose anchor byte is < X.
__device__ __forceinline__ int64_t tokens_before(const Row &r, int64_t X, int32_t k, int32_t cls) {
    int64_t c = 0;
    if (X > r.off) {
        // body anchors off + j*k < X  <=>  j < ceil((X - off) / k)
        c += (X >= r.end) ? r.nb : (X - r.off + k - 1) / k;
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
// validity bits (bit 31 = first byte) for the A/C/G/T/a/c/g/t test.
__device__ __forceinline__ void classify16(uint4 v, uint32_t &code, uint32_t &valid) {
    uint32_t x[4] = {v.x, v.y, v.z, v.w};
    code = 0;
    valid = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t f = x[q] | 0x20202020u;  // fold case: only A/a (etc.) map to a (etc.)
        uint32_t d = ((f >> 1) ^ (f >> 2)) & 0x03030303u;  // a->0 c->1 g->2 t->3
        auto nz = [](uint32_t z) { return ((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z; };
        uint32_t hit = ~(nz(f ^ 0x61616161u) & nz(f ^ 0x63636363u) & nz(f ^ 0x67676767u) & nz(f ^ 0x74747474u)) &
                       0x80808080u;
        // digits of bytes 0..3 -> 8 bits, byte 0 most significant
        uint32_t r = __builtin_bswap32(d);
        uint32_t t = r | (r >> 6);
        uint32_t p = (t & 0xFu) | ((t >> 12) & 0xF0u);
        code |= p << (24 - 8 * q);
        // validity bits of bytes 0..3 -> 4 bits, byte 0 most significant
        uint32_t vb = ((hit >> 7) * 0x80402010u) >> 28;
        valid |= vb << (28 - 4 * q);
    }
}

__device__ __forceinline__ uint4 load_chunk(const EncodeArgs &a, int64_t q0) {
    if (q0 >= a.shift && q0 + 16 <= a.shift + a.nbytes)
        return *reinterpret_cast<const uint4 *>(a.abase + q0);
    uint32_t w[4] = {0, 0, 0, 0};
    for (int b = 0; b < 16; ++b) {
        int64_t qb = q0 + b;
        if (qb >= a.shift && qb < a.shift + a.nbytes) w[b >> 2] |= (uint32_t)a.abase[qb] << (8 * (b & 3));
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

template <bool KMER>
__global__ __launch_bounds__(NT) void k_encode(EncodeArgs a) {
    extern __shared__ __align__(16) uint8_t dyn[];
    __shared__ int32_t lut_s[256];
    __shared__ int64_t s_off[NT], s_end[NT], s_nb[NT], s_clo[NT], s_chi[NT], s_dlo[NT], s_gpre[NT];
    __shared__ int64_t s_tmp[NT / dev::kWave + 1];
    __shared__ int64_t s_ticket, s_ia, s_ib, s_excl;
    __shared__ uint32_t s_err;

    const int tid = threadIdx.x;
    if (!KMER)
        for (int i = tid; i < 256; i += NT) lut_s[i] = a.lut[i];
    const uint32_t parity = dev::ld_relaxed32(a.q.hdr + 2);
    uint64_t *st = parity ? a.q.status1 : a.q.status0;
    uint64_t *st_other = parity ? a.q.status0 : a.q.status1;
    const int64_t B = a.tileB;
    const int64_t nchunks = B / 16 + 1;
    uint32_t *codes = reinterpret_cast<uint32_t *>(dyn);
    uint32_t *valid = codes + nchunks;
    uint8_t *raw = dyn;
    const int32_t k = KMER ? a.k : 1;
    const int64_t al = (int64_t)((reinterpret_cast<uintptr_t>(a.ids) >> 2) & 3);

    for (;;) {
        if (tid == 0) {
            s_ticket = (int64_t)atomicAdd(a.q.hdr + 0, 1u);
            s_err = 0;
        }
        __syncthreads();
        const int64_t t = s_ticket;
        if (t >= a.ntiles) break;
        uint32_t err = 0;

        // Housekeeping shares: zero the other parity's status words for the
        // next launch, and check a strided slice of the offsets.
        for (int64_t j = t + (int64_t)tid * a.ntiles; j < a.q.clear_n; j += (int64_t)NT * a.ntiles) st_other[j] = 0;
        for (int64_t i = t + (int64_t)tid * a.ntiles; i < a.n; i += (int64_t)NT * a.ntiles) {
            int64_t o0 = a.offs[i], o1 = a.offs[i + 1];
            if (o0 < 0 || o1 < o0 || o1 > a.nbytes) err |= DNATOK_DERR_OFFSETS;
        }

        const int64_t P0 = t * B - a.shift;
        const int64_t P1 = (t == a.ntiles - 1) ? INT64_MAX : P0 + B;

        // Stage the tile (and one halo chunk) into LDS.
        for (int64_t m = tid; m < nchunks; m += NT) {
            uint4 v = load_chunk(a, t * B + 16 * m);
            if (KMER) {
                uint32_t c, vb;
                classify16(v, c, vb);
                codes[m] = c;
                valid[m] = vb;
            } else {
                reinterpret_cast<uint4 *>(raw)[m] = v;
            }
        }

        // Rows with an anchor in [P0, P1): [ia, ib).
        if (tid == 0) {
            int64_t lo = 0, hi = a.n;
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                int64_t o0 = a.offs[mid], o1 = a.offs[mid + 1];
                int64_t last = (o1 > o0) ? o1 - 1 : o0;
                if (last >= P0) hi = mid;
                else lo = mid + 1;
            }
            int64_t ia = lo;
            hi = a.n;
            if (P1 != INT64_MAX) {
                while (lo < hi) {
                    int64_t mid = (lo + hi) >> 1;
                    if (a.offs[mid] >= P1) hi = mid;
                    else lo = mid + 1;
                }
            } else {
                lo = a.n;
            }
            s_ia = ia;
            s_ib = lo;
        }
        __syncthreads();
        const int64_t ia = s_ia, ib = s_ib;

        auto load_row = [&](int64_t i) {
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

        // Count pass: tokens owned by this tile.
        int64_t agg = 0;
        for (int64_t cb = ia; cb < ib; cb += NT) {
            int64_t i = cb + tid;
            int64_t cnt = 0;
            if (i < ib) {
                Row r = load_row(i);
                cnt = tokens_before(r, P1, k, a.cls) - tokens_before(r, P0, k, a.cls);
            }
            agg += dev::block_sum<NT>(cnt, s_tmp);
        }
        if (tid == 0) s_excl = dev::lookback(st, t, agg);
        __syncthreads();

        // Write pass, one chunk of up to NT rows at a time.
        int64_t tokbase = s_excl;
        for (int64_t cb = ia; cb < ib; cb += NT) {
            const int64_t i = cb + tid;
            const int nrows = (int)((ib - cb) < NT ? (ib - cb) : NT);
            int64_t tcnt = 0, gcnt = 0, clo = 0, chi = 0, dlo = 0;
            Row r = {0, 0, 0, 0};
            if (i < ib) {
                r = load_row(i);
                int64_t tlo = tokens_before(r, P0, k, a.cls), thi = tokens_before(r, P1, k, a.cls);
                tcnt = thi - tlo;
                if (a.padded && r.len > a.W) {
                    err |= DNATOK_DERR_ROW_WIDTH;
                } else {
                    clo = cells_before(r, P0, k, a.cls, a.padded, a.left, a.W);
                    chi = cells_before(r, P1, k, a.cls, a.padded, a.left, a.W);
                }
            }
            int64_t tot;
            int64_t pre = dev::block_excl_scan<NT>(tcnt, s_tmp, &tot);
            if (i < ib) {
                if (r.off >= P0 && r.off < P1) a.out_offs[i] = a.base + tokbase + pre;
                dlo = a.padded ? i * a.W + clo : tokbase + pre;
                if (chi > clo) gcnt = ((dlo + al + (chi - clo) - 1) >> 2) - ((dlo + al) >> 2) + 1;
            }
            int64_t G;
            int64_t gpre = dev::block_excl_scan<NT>(gcnt, s_tmp, &G);
            if (i < ib) {
                s_off[tid] = r.off;
                s_end[tid] = r.end;
                s_nb[tid] = r.nb;
                s_clo[tid] = clo;
                s_chi[tid] = chi;
                s_dlo[tid] = dlo;
                s_gpre[tid] = gpre;
            }
            __syncthreads();

            int s = 0;
            for (int64_t qi = tid; qi < G; qi += NT) {
                // segment holding group qi: the last s with gpre[s] <= qi
                if (!(s_gpre[s] <= qi && (s + 1 >= nrows || s_gpre[s + 1] > qi))) {
                    int lo = 0, hi = nrows - 1;
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (s_gpre[mid] <= qi) lo = mid;
                        else hi = mid - 1;
                    }
                    s = lo;
                }
                const int64_t off = s_off[s], end = s_end[s], nb = s_nb[s];
                const int64_t len = nb + 2 * a.cls;
                const int64_t sclo = s_clo[s], schi = s_chi[s], sdlo = s_dlo[s];
                const int64_t eb = (((sdlo + al) >> 2) + (qi - s_gpre[s])) * 4 - al;
                const int64_t lead = (a.padded && a.left) ? a.W - len : 0;
                int32_t v[4];
                uint32_t mk = 0;
                bool in[4];
                bool all_in = true;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int64_t e = eb + rr;
                    const int64_t c = sclo + (e - sdlo);
                    in[rr] = (c >= sclo && c < schi);
                    if (in[rr] && !a.padded && e >= a.cap) {
                        in[rr] = false;
                        err |= DNATOK_DERR_CAPACITY;
                    }
                    all_in = all_in && in[rr];
                    int32_t val = a.pad_id;
                    uint32_t m = 0;
                    const int64_t tt = c - lead;
                    if (in[rr] && tt >= 0 && tt < len) {
                        m = 1;
                        if (a.cls && tt == 0) {
                            val = a.cls_id;
                        } else if (a.cls && tt == len - 1) {
                            val = a.sep_id;
                        } else {
                            const int64_t j = tt - a.cls;
                            if (KMER) {
                                const int64_t p = off + j * k;
                                if (p + k > end) {
                                    val = DNATOK_ID_UNK;
                                } else {
                                    const int64_t idx = p - P0;
                                    const int64_t w = idx >> 4;
                                    const int o = (int)(idx & 15);
                                    const uint64_t c64 = ((uint64_t)codes[w] << 32) | codes[w + 1];
                                    const uint32_t digits = (uint32_t)((c64 << (2 * o)) >> (64 - 2 * k));
                                    const uint32_t v32 = valid[w] | (valid[w + 1] >> 16);
                                    const uint32_t okb = (v32 << o) >> (32 - k);
                                    val = (okb == ((1u << k) - 1)) ? (int32_t)(5 + digits) : DNATOK_ID_UNK;
                                }
                            } else {
                                val = lut_s[raw[off + j - P0]];
                            }
                        }
                    }
                    v[rr] = val;
                    mk |= m << (8 * rr);
                }
                int32_t *dst = a.ids + eb;
                if (all_in) {
                    *reinterpret_cast<int4 *>(dst) = make_int4(v[0], v[1], v[2], v[3]);
                    if (a.padded) {
                        int8_t *md = a.mask + eb;
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
                        dst[rr] = v[rr];
                        if (a.padded) a.mask[eb + rr] = (int8_t)((mk >> (8 * rr)) & 1);
                    }
                }
            }
            __syncthreads();
            tokbase += tot;
        }
        if (t == a.ntiles - 1 && tid == 0) a.out_offs[a.n] = a.base + s_excl + agg;
        if (err) atomicOr(&s_err, err);
        __syncthreads();
        if (tid == 0 && s_err) dev::raise_error(a.q.hdr, s_err);
    }
    if (tid == 0) dev::finish_block(a.q.hdr);
}

}  // namespace

int launch_encode(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                  int32_t n, int32_t *d_ids, int64_t cap, int64_t *d_out_offsets, int8_t *d_mask,
                  const dnatok_encode_opts &o, hipStream_t stream) {
    const bool kmer = (v->kind == DNATOK_KMER);
    const int64_t B = kmer ? 16384 : 8192;
    EncodeArgs a;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(d_bytes);
    a.shift = (int64_t)(addr & 15);
    a.abase = d_bytes ? d_bytes - a.shift : nullptr;
    a.nbytes = nbytes;
    a.offs = d_offsets;
    a.n = n;
    a.k = kmer ? v->k : 1;
    a.ids = d_ids;
    a.cap = cap;
    a.out_offs = d_out_offsets;
    a.mask = d_mask;
    a.lut = v->d_lut;
    a.cls = o.add_cls_sep ? 1 : 0;
    a.padded = (o.layout == DNATOK_PADDED) ? 1 : 0;
    a.left = (o.pad_side == DNATOK_PAD_LEFT) ? 1 : 0;
    a.pad_id = v->pad_id;
    a.cls_id = v->cls_id;
    a.sep_id = v->sep_id;
    a.W = a.padded ? o.pad_to : 0;
    a.base = o.offset_base;
    a.tileB = B;
    a.ntiles = (nbytes + a.shift) / B + 1;

    Workspace *ws = nullptr;
    int rc = get_workspace(stream, a.ntiles, &ws);
    if (rc) return rc;
    a.q.hdr = ws->d_hdr;
    a.q.status0 = ws->d_status;
    a.q.status1 = ws->d_status + ws->cap;
    if (a.ntiles > ws->high_water) ws->high_water = a.ntiles;
    a.q.clear_n = ws->high_water;

    const size_t dyn = kmer ? (size_t)(B / 16 + 1) * 8 : (size_t)(B / 16 + 1) * 16;
    int per_cu = 0;
    if (kmer)
        DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_encode<true>, NT, dyn));
    else
        DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_encode<false>, NT, dyn));
    if (per_cu < 1) per_cu = 1;
    int64_t grid = (int64_t)device_cu_count() * per_cu;
    if (grid > a.ntiles) grid = a.ntiles;
    if (kmer)
        hipLaunchKernelGGL(k_encode<true>, dim3((unsigned)grid), dim3(NT), dyn, stream, a);
    else
        hipLaunchKernelGGL(k_encode<false>, dim3((unsigned)grid), dim3(NT), dyn, stream, a);
    DNATOK_HIP(hipGetLastError());
    return DNATOK_OK;
}

}  // namespace dnatok
