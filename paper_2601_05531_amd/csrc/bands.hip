// PADDED encode by row bands (SINGLE, LUT256, KMER; several k-mer
// vocabularies in one pass).
//
// Paper: the bytes branch of the EmbedFromStrings algorithm produces an
// equal-width B x T' id matrix (MapKmer or the table lookup, then padding to
// token_len); Design, "Encoding paths", bytes path.
//
// In a PADDED output every row owns W consecutive cells per vocabulary, so
// the cells of R consecutive rows form one contiguous region of each output.
// A workgroup takes such a band: it reads the band's bytes once into LDS
// (k-mer kinds classified into 2-bit digits and validity bits on the way,
// table kinds kept as bytes) and then writes every cell of the band for
// every vocabulary, four cells per 16-byte store. Each cell follows from its
// row and column alone (CLS, body token, short final frame, SEP or pad), so
// there is no segment pass, no scan and no edge pass. Bands are small (a
// few KiB of input), there are many more of them than resident workgroups,
// and consecutive bands go to consecutive XCDs: workgroups that start late
// load while others write, and every XCD writes everywhere in the output.
//
// The host sizes R from pad_to so that a band's bytes fit its LDS stage.
// Offsets the device finds invalid (or a row longer than pad_to allows) can
// make a band's span exceed the stage; such a band reads its bytes from
// global memory cell by cell (same ids, slower).
#include "common.hpp"
#include "device.hpp"
#include "rowscan.hpp"

namespace dnatok {

namespace {

constexpr int NTB = 256;
constexpr int kBandVocabs = 8;
constexpr int kMaxBandRows = 64;

struct BandVocab {
    int32_t k;
    int32_t al;  // element misalignment of ids within 16 bytes
    int32_t *ids;
    int8_t *mask;
    int64_t W;
    uint32_t winv;  // floor((2^32 - 1) / W), W < 2^31
    int32_t pad_id, cls_id, sep_id;
};

struct BandArgs {
    const uint8_t *abase;  // input base aligned down to 16 bytes
    int64_t shift;         // d_bytes - abase
    int64_t nbytes;
    const int64_t *offs;
    int32_t n;
    int32_t nv;
    int32_t cls, left;
    int32_t R;             // rows per band
    int32_t stage_chunks;  // 16-byte chunks the LDS stage holds
    int64_t nbands;
    int32_t lead;          // blocks before the bands (fused row scans, then idle)
    int32_t nscan;
    const int32_t *lut;
    uint32_t *err_hdr;
    BandVocab vo[kBandVocabs];
    RowScanArgs scan[kBandVocabs];
};

__device__ __forceinline__ uint32_t umod_w(uint32_t x, uint32_t W, uint32_t winv, uint32_t *q) {
    uint32_t d = __umulhi(x, winv);
    uint32_t r = x - d * W;
    if (r >= W) {
        r -= W;
        ++d;
    }
    *q = d;
    return r;
}

// Digits (most significant first) and validity of k bytes read one by one
// from global memory, positions clamped to the input (slow path).
__device__ __forceinline__ int32_t kmer_global(const BandArgs &a, int64_t pos, int32_t k) {
    uint32_t v = 0;
    bool ok = true;
    for (int32_t j = 0; j < k; ++j) {
        const int64_t p = pos + j;
        const uint8_t b = (p >= 0 && p < a.nbytes) ? a.abase[a.shift + p] : 0;
        const uint8_t f = b | 0x20;
        const int32_t d = f == 'a' ? 0 : f == 'c' ? 1 : f == 'g' ? 2 : f == 't' ? 3 : -1;
        ok = ok && d >= 0;
        v = (v << 2) | (uint32_t)(d & 3);
    }
    return ok ? (int32_t)(5 + v) : DNATOK_ID_UNK;
}

// Ids of k-mers from the staged windows (as the tile kernel stages them):
// win64[m] holds the digits of chunks m and m + 1, val32[m] their validity.
__device__ __forceinline__ int32_t kmer_lds(const uint64_t *win64, const uint32_t *val32, uint32_t idx, int32_t k) {
    const uint32_t w = idx >> 4, o = idx & 15;
    const uint32_t digits = (uint32_t)(win64[w] >> (64 - 2 * (o + (uint32_t)k))) & ((1u << (2 * k)) - 1);
    const uint32_t km = (1u << k) - 1;
    const bool ok = ((val32[w] >> (32 - o - (uint32_t)k)) & km) == km;
    return ok ? (int32_t)(5 + digits) : DNATOK_ID_UNK;
}

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Four consecutive k-mers (k <= 8) from staged byte idx0 on.
__device__ __forceinline__ i32x4 kmer4_lds(const uint64_t *win64, const uint32_t *val32, uint32_t idx0, int32_t k) {
    const uint32_t w = idx0 >> 4, o = idx0 & 15;
    const uint64_t w0 = win64[w], w1 = win64[w + 1];
    const uint32_t v0 = val32[w], v1 = val32[w + 1];
    const uint64_t X = (w0 << (2 * o)) | (((uint64_t)(uint32_t)w1 << (2 * o)) >> 32);
    const uint32_t nV = ~(uint32_t)((((uint64_t)v0 << 32) | (uint64_t)(v1 << 16)) << o >> 32);
    const uint32_t dm = (1u << (2 * k)) - 1u;
    i32x4 r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t sh = 64u - 2u * (uint32_t)(k * (q + 1));
        const uint32_t vm = ((1u << k) - 1u) << (32 - k * (q + 1));
        const int32_t id = 5 + (int32_t)((uint32_t)(X >> sh) & dm);
        r[q] = (nV & vm) == 0 ? id : DNATOK_ID_UNK;
    }
    return r;
}

template <bool KMER>
__global__ __launch_bounds__(NTB) void k_bands(BandArgs a) {
    extern __shared__ __align__(16) uint8_t dyn[];
    __shared__ int64_t s_o0[kMaxBandRows], s_o1[kMaxBandRows];
    __shared__ int32_t s_nb[kBandVocabs * kMaxBandRows];   // body tokens of (vocabulary, row)
    __shared__ uint32_t s_ro[kMaxBandRows];                // staged index of each row's first byte
    __shared__ int32_t s_lut[256];
    __shared__ int64_t s_lo, s_hi;
    __shared__ int64_t s_tmp[NTB / dev::kWave + 1];
    const int tid = threadIdx.x;
    if ((int)blockIdx.x < a.lead) {
        if ((int)blockIdx.x < a.nscan) rowscan_single_block(a.scan[blockIdx.x], s_tmp, a.err_hdr);
        return;
    }
    const int64_t band = (int64_t)blockIdx.x - a.lead;
    const int64_t r0 = band * a.R;
    const int nr = (int)min((int64_t)a.R, (int64_t)a.n - r0);
    if (!KMER) s_lut[tid] = a.lut[tid];
    // row byte ranges, validated and clamped as the row scan does
    if (tid < nr) {
        int64_t o0 = a.offs[r0 + tid], o1 = a.offs[r0 + tid + 1];
        o0 = o0 < 0 ? 0 : (o0 > a.nbytes ? a.nbytes : o0);
        o1 = o1 < o0 ? o0 : (o1 > a.nbytes ? a.nbytes : o1);
        s_o0[tid] = o0;
        s_o1[tid] = o1;
    }
    __syncthreads();
    if (tid < dev::kWave) {
        int64_t lo = INT64_MAX, hi = 0;
        for (int i = tid; i < nr; i += dev::kWave) {
            lo = min(lo, s_o0[i]);
            hi = max(hi, s_o1[i]);
        }
#pragma unroll
        for (int d = dev::kWave / 2; d > 0; d >>= 1) {
            lo = min(lo, (int64_t)__shfl_xor(lo, d, dev::kWave));
            hi = max(hi, (int64_t)__shfl_xor(hi, d, dev::kWave));
        }
        if (tid == 0) {
            s_lo = lo == INT64_MAX ? 0 : lo;
            s_hi = hi;
        }
    }
    __syncthreads();
    // the band's bytes in abase coordinates [q0, q1), staged from chunk c0 on
    const int64_t q0 = s_lo + a.shift, q1 = max(s_hi, s_lo) + a.shift;
    const int64_t c0 = q0 >> 4;
    const int64_t nch = ((q1 + 15) >> 4) - c0 + 2;  // two spare chunks: a window reads the next two
    const bool staged = nch <= a.stage_chunks;
    uint64_t *win64 = reinterpret_cast<uint64_t *>(dyn);
    uint32_t *val32 = reinterpret_cast<uint32_t *>(win64 + a.stage_chunks);
    uint8_t *raw = dyn;
    if (staged) {
        // all of this thread's chunk loads first (in bounds: whole 16-byte
        // vectors inside the input, else byte by byte), then classify
        const int64_t lim = a.shift + a.nbytes;
        for (int64_t m0 = 0; m0 < nch; m0 += 4 * NTB) {
            uint4 x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t m = m0 + u * NTB + tid;
                const int64_t q = (c0 + m) << 4;
                if (m < nch && q >= a.shift && q + 16 <= lim) {
                    const u32x4 t = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(a.abase + q));
                    x[u] = make_uint4(t[0], t[1], t[2], t[3]);
                } else {
                    uint32_t w[4] = {0, 0, 0, 0};
                    if (m < nch)
                        for (int b = 0; b < 16; ++b)
                            if (q + b >= a.shift && q + b < lim) w[b >> 2] |= (uint32_t)a.abase[q + b] << (8 * (b & 3));
                    x[u] = make_uint4(w[0], w[1], w[2], w[3]);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t m = m0 + u * NTB + tid;
                if (m >= nch) continue;
                if (KMER) {
                    uint32_t c, vb;
                    dev::classify16(x[u], c, vb);
                    uint32_t *w32 = reinterpret_cast<uint32_t *>(win64);
                    uint16_t *v16 = reinterpret_cast<uint16_t *>(val32);
                    w32[2 * m + 1] = c;
                    v16[2 * m + 1] = (uint16_t)(vb >> 16);
                    if (m > 0) {
                        w32[2 * m - 2] = c;
                        v16[2 * m - 2] = (uint16_t)(vb >> 16);
                    }
                } else {
                    reinterpret_cast<uint4 *>(raw)[m] = x[u];
                }
            }
        }
        if (KMER && tid == 0) {  // low half of the last window
            reinterpret_cast<uint32_t *>(win64)[2 * (nch - 1)] = 0;
            reinterpret_cast<uint16_t *>(val32)[2 * (nch - 1)] = 0;
        }
    }
    const int64_t sbase = c0 << 4;  // abase position of staged byte 0
    if (tid < nr) s_ro[tid] = (uint32_t)(s_o0[tid] + a.shift - sbase);
    for (int t = tid; t < a.nv * nr; t += NTB) {
        const int vi = t / nr, r = t - vi * nr;
        const int64_t L = s_o1[r] - s_o0[r];
        const int32_t k = KMER ? a.vo[vi].k : 1;
        s_nb[vi * kMaxBandRows + r] = (int32_t)(KMER ? div_k(L + k - 1, k, 0xFFFFFFFFu / (uint32_t)k) : L);
    }
    __syncthreads();

    for (int vi = 0; vi < a.nv; ++vi) {
        const BandVocab &o = a.vo[vi];
        const int32_t k = KMER ? o.k : 1;
        const int64_t W = o.W;
        const int64_t E0 = r0 * W, E1 = E0 + (int64_t)nr * W;  // this band's cells
        const int64_t g0 = (E0 + o.al) >> 2, g1 = (E1 - 1 + o.al) >> 2;
        const bool mask4 = ((reinterpret_cast<uintptr_t>(o.mask) - (uintptr_t)o.al) & 3) == 0;
        // id and mask of band cell f (row f / W, column f % W); m = 2 marks a
        // row too long for pad_to, which writes nothing (the row scan raised
        // the flag). body4: this cell and the next three are full body
        // tokens of one row, the first at staged byte idx.
        const int32_t W32 = (int32_t)W;
        const int32_t *nbv = s_nb + vi * kMaxBandRows;
        auto cell = [&](uint32_t f, int32_t &id, uint32_t &m, bool &body4, uint32_t &idx) {
            uint32_t r;
            const int32_t c = (int32_t)umod_w(f, (uint32_t)W, o.winv, &r);
            const int32_t nb = nbv[r];
            const int32_t len = nb + 2 * a.cls;
            const int32_t tt = c - (a.left ? W32 - len : 0);
            id = o.pad_id;
            m = 0;
            body4 = false;
            idx = 0;
            if (len > W32) {
                m = 2;
                return;
            }
            if (tt < 0 || tt >= len) return;
            m = 1;
            if (a.cls && tt == 0) {
                id = o.cls_id;
            } else if (a.cls && tt == len - 1) {
                id = o.sep_id;
            } else {
                const int32_t j = tt - a.cls;
                const int64_t L = s_o1[r] - s_o0[r];
                const bool tail = KMER && (int64_t)nb * k != L;
                if (tail && j == nb - 1) {
                    id = DNATOK_ID_UNK;
                } else if (staged) {
                    idx = s_ro[r] + (uint32_t)(j * k);
                    id = KMER ? kmer_lds(win64, val32, idx, k) : s_lut[raw[idx]];
                    body4 = j + 4 <= nb - (tail ? 1 : 0);
                } else {
                    const int64_t pos = s_o0[r] + (int64_t)j * k;
                    id = KMER ? kmer_global(a, pos, k) : s_lut[a.abase[a.shift + pos]];
                }
            }
        };
        for (int64_t g = g0 + tid; g <= g1; g += NTB) {
            const int64_t e = 4 * g - o.al;
            int32_t v[4];
            uint32_t mk = 0;
            bool in[4], all_in = true;
            const bool inside = e >= E0 && e + 3 < E1;
            int32_t id0 = 0;
            uint32_t m0 = 0, idx0 = 0;
            bool b4 = false;
            if (inside) cell((uint32_t)(e - E0), id0, m0, b4, idx0);
            if (b4 && (!KMER || k <= 8)) {
                // four body tokens of one row from one staged read
                if (KMER) {
                    const i32x4 y = kmer4_lds(win64, val32, idx0, k);
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = y[q];
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = s_lut[raw[idx0 + q]];
                }
                mk = 0x01010101u;
#pragma unroll
                for (int q = 0; q < 4; ++q) in[q] = true;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t eq = e + q;
                    in[q] = eq >= E0 && eq < E1;
                    v[q] = o.pad_id;
                    if (!in[q]) {
                        all_in = false;
                        continue;
                    }
                    int32_t id;
                    uint32_t m, ix;
                    bool bb;
                    if (q == 0 && inside) {
                        id = id0;
                        m = m0;
                    } else {
                        cell((uint32_t)(eq - E0), id, m, bb, ix);
                    }
                    if (m == 2) {
                        in[q] = false;
                        all_in = false;
                        continue;
                    }
                    v[q] = id;
                    mk |= m << (8 * q);
                }
            }
            int32_t *dst = o.ids + e;
            if (all_in) {
                __builtin_nontemporal_store(i32x4{v[0], v[1], v[2], v[3]}, reinterpret_cast<i32x4 *>(dst));
                if (mask4)
                    __builtin_nontemporal_store(mk, reinterpret_cast<uint32_t *>(o.mask + e));
                else
                    for (int q = 0; q < 4; ++q) o.mask[e + q] = (int8_t)((mk >> (8 * q)) & 1);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (!in[q]) continue;
                    dst[q] = v[q];
                    o.mask[e + q] = (int8_t)((mk >> (8 * q)) & 1);
                }
            }
        }
    }
}

template <bool KMER>
int band_occupancy(size_t dyn, int *per_cu) {
    DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_bands<KMER>, NTB, dyn));
    return DNATOK_OK;
}

}  // namespace

// PADDED encode by row bands; returns DNATOK_OK having launched, or a
// negative code. *used is false (and nothing is launched) when the batch does
// not suit bands (a row could exceed the largest stage).
int launch_encode_bands(const dnatok_vocab *const *vs, int nv, const uint8_t *d_bytes, int64_t nbytes,
                        const int64_t *d_offsets, int32_t n, int32_t *const *d_ids, const int64_t *caps,
                        int8_t *const *d_masks, const dnatok_encode_opts *os, int64_t stage_bytes,
                        int64_t *const *d_out_offsets, hipStream_t stream, bool *used) {
    *used = false;
    if (nv < 1 || nv > kBandVocabs) return DNATOK_OK;
    const dnatok_vocab *v = vs[0];
    const bool kmer = (v->kind == DNATOK_KMER);
    const dnatok_encode_opts &o = os[0];
    if (o.layout != DNATOK_PADDED || o.variant) return DNATOK_OK;
    BandArgs a = {};
    a.cls = o.add_cls_sep ? 1 : 0;
    a.left = (o.pad_side == DNATOK_PAD_LEFT) ? 1 : 0;
    // longest row any vocabulary's pad_to admits, in bytes
    int64_t maxrow = INT64_MAX;
    for (int vi = 0; vi < nv; ++vi) {
        const int64_t k = kmer ? vs[vi]->k : 1;
        const int64_t W = os[vi].pad_to;
        if (W >= (1ll << 31)) return DNATOK_OK;
        maxrow = std::min(maxrow, std::max<int64_t>(0, W - 2 * a.cls) * k);
    }
    if (maxrow > stage_bytes) return DNATOK_OK;
    int64_t R = maxrow > 0 ? stage_bytes / maxrow : kMaxBandRows;
    R = std::max<int64_t>(1, std::min<int64_t>(R, kMaxBandRows));
    if (n > 0 && (int64_t)n < R) R = n;
    // a band's cells are indexed in 32 bits
    int64_t Wmax = 0;
    for (int vi = 0; vi < nv; ++vi) Wmax = std::max<int64_t>(Wmax, os[vi].pad_to);
    while (R > 1 && R * Wmax >= (1ll << 31)) R >>= 1;
    if (R * Wmax >= (1ll << 31)) return DNATOK_OK;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(d_bytes);
    a.shift = (int64_t)(addr & 15);
    a.abase = d_bytes ? d_bytes - a.shift : nullptr;
    a.nbytes = nbytes;
    a.offs = d_offsets;
    a.n = n;
    a.nv = nv;
    a.R = (int32_t)R;
    // a band of valid rows spans at most R * maxrow bytes: its chunks plus
    // the partial ones at both ends and the two spare ones
    a.stage_chunks = (int32_t)((R * std::max<int64_t>(maxrow, 1) + 15) / 16 + 4);
    a.nbands = n > 0 ? (n + R - 1) / R : 0;
    a.lut = v->d_lut;
    Workspace *ws = nullptr;
    int rc = get_workspace(stream, 1, &ws);
    if (rc) return rc;
    a.err_hdr = ws->d_hdr;
    const bool fuse = n <= 16384;
    a.nscan = fuse ? nv : 0;
    a.lead = fuse ? 8 : 0;
    for (int vi = 0; vi < nv; ++vi) {
        BandVocab &bv = a.vo[vi];
        bv.k = kmer ? vs[vi]->k : 1;
        bv.al = (int32_t)((reinterpret_cast<uintptr_t>(d_ids[vi]) >> 2) & 3);
        bv.ids = d_ids[vi];
        bv.mask = d_masks[vi];
        bv.W = os[vi].pad_to;
        bv.winv = (uint32_t)(0xFFFFFFFFull / (uint64_t)bv.W);
        bv.pad_id = vs[vi]->pad_id;
        bv.cls_id = vs[vi]->cls_id;
        bv.sep_id = vs[vi]->sep_id;
        (void)caps;
        RowScanSpec sp;
        sp.offs = d_offsets;
        sp.n = n;
        sp.nbytes = nbytes;
        sp.out = d_out_offsets[vi];
        sp.k = bv.k;
        sp.kmer = kmer ? 1 : 0;
        sp.overlap = 0;
        sp.cls = a.cls;
        sp.padded = 1;
        sp.W = bv.W;
        sp.base = os[vi].offset_base;
        if (fuse) {
            RowScanArgs &s = a.scan[vi];
            s.offs = d_offsets;
            s.n = n;
            s.nbytes = nbytes;
            s.out_offs = d_out_offsets[vi];
            s.k = bv.k;
            s.kinv = 0xFFFFFFFFu / (uint32_t)bv.k;
            s.kmer = kmer ? 1 : 0;
            s.overlap = 0;
            s.cls = a.cls;
            s.padded = 1;
            s.W = bv.W;
            s.base = os[vi].offset_base;
            s.nunits = std::max<int64_t>(1, ((int64_t)n + kUnitRows - 1) / kUnitRows);
        } else {
            rc = launch_rowscan_spec(sp, stream);
            if (rc) return rc;
        }
    }
    const size_t dyn = kmer ? (size_t)a.stage_chunks * 12 : (size_t)a.stage_chunks * 16;
    if (dyn > 64 * 1024) {
        DNATOK_HIP(hipFuncSetAttribute(kmer ? (const void *)k_bands<true> : (const void *)k_bands<false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    }
    const int64_t grid = a.lead + a.nbands;
    if (grid > 0) {
        if (kmer)
            hipLaunchKernelGGL(k_bands<true>, dim3((unsigned)grid), dim3(NTB), dyn, stream, a);
        else
            hipLaunchKernelGGL(k_bands<false>, dim3((unsigned)grid), dim3(NTB), dyn, stream, a);
        DNATOK_HIP(hipGetLastError());
    }
    *used = true;
    return DNATOK_OK;
}

}  // namespace dnatok
