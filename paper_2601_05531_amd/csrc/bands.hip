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
    int32_t overlap;       // KMER: stride-1 windows (L - k + 1 of them; one UNK for 0 < L < k)
    int32_t revcomp;       // encode each row's reverse complement
    int32_t R;             // rows per band
    int32_t P;             // parts per row (P > 1: R = 1, part p takes the tokens starting in bytes [pU, (p+1)U))
    int64_t U;             // bytes per part
    int32_t kmax;          // the longest k among the vocabularies (a part stages U + kmax bytes)
    int32_t stage_chunks;  // 16-byte chunks the LDS stage holds
    int64_t nbands;
    int32_t lead;          // blocks before the bands (fused row scans, then idle)
    int32_t nscan;
    const int32_t *lut;
    uint32_t *err_hdr;
    BandVocab vo[kBandVocabs];
    RowScanArgs scan[kBandVocabs];
};

// Digits (most significant first) of k bytes read one by one from global
// memory, positions clamped to the input (slow path); -1 if any byte is not
// A/C/G/T in either case.
__device__ __forceinline__ int64_t kmer_global(const BandArgs &a, int64_t pos, int32_t k) {
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
    return ok ? (int64_t)v : -1;
}

// The k 2-bit digits of v in reverse order (k <= 16).
__device__ __forceinline__ uint32_t rev_digits(uint32_t v, int32_t k) {
    uint32_t r = __builtin_bitreverse32(v);
    r = ((r >> 1) & 0x55555555u) | ((r & 0x55555555u) << 1);
    return r >> (32 - 2 * k);
}

// Id of a k-mer whose forward digits are fv (or -1: a byte outside ACGT);
// the reverse complement reverses and complements the digits.
__device__ __forceinline__ int32_t kmer_id(int64_t fv, int32_t k, bool rc) {
    if (fv < 0) return DNATOK_ID_UNK;
    const uint32_t dm = (1u << (2 * k)) - 1u;
    return 5 + (int32_t)(rc ? (rev_digits((uint32_t)fv, k) ^ dm) : (uint32_t)fv);
}

__device__ __forceinline__ uint32_t complement_byte(uint32_t b) {
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

// Forward digits of the k-mer at staged byte idx (staged windows as the
// tile kernel stages them: win64[m] holds the digits of chunks m and m + 1,
// val32[m] their validity), or -1 if a byte is not A/C/G/T.
__device__ __forceinline__ int64_t kmer_lds(const uint64_t *win64, const uint32_t *val32, uint32_t idx, int32_t k) {
    const uint32_t w = idx >> 4, o = idx & 15;
    const uint32_t digits = (uint32_t)(win64[w] >> (64 - 2 * (o + (uint32_t)k))) & ((1u << (2 * k)) - 1);
    const uint32_t km = (1u << k) - 1;
    const bool ok = ((val32[w] >> (32 - o - (uint32_t)k)) & km) == km;
    return ok ? (int64_t)digits : -1;
}

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Four ids from the 32 staged bases starting at byte idx0: id q is the
// k-mer whose forward digits start at base p0 + q * dp of that window
// (p0 + 3 * dp + k <= 32), reverse complemented if rc.
__device__ __forceinline__ i32x4 kmer4_lds(const uint64_t *win64, const uint32_t *val32, uint32_t idx0, int32_t k,
                                           int32_t p0, int32_t dp, bool rc) {
    const uint32_t w = idx0 >> 4, o = idx0 & 15;
    const uint64_t w0 = win64[w], w1 = win64[w + 1];
    const uint32_t v0 = val32[w], v1 = val32[w + 1];
    const uint64_t X = (w0 << (2 * o)) | (((uint64_t)(uint32_t)w1 << (2 * o)) >> 32);
    const uint32_t nV = ~(uint32_t)((((uint64_t)v0 << 32) | (uint64_t)(v1 << 16)) << o >> 32);
    const uint32_t dm = (1u << (2 * k)) - 1u;
    const uint32_t km = (1u << k) - 1u;
    i32x4 r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int32_t p = p0 + q * dp;
        const uint32_t fv = (uint32_t)(X >> (64 - 2 * (p + k))) & dm;
        const bool bad = ((nV >> (32 - p - k)) & km) != 0;
        r[q] = bad ? DNATOK_ID_UNK : 5 + (int32_t)(rc ? (rev_digits(fv, k) ^ dm) : fv);
    }
    return r;
}

// Row scan of one vocabulary's token counts by one workgroup (the fused
// PADDED case, a few thousand rows), four rows per thread per pass: the same
// validation and totals as the stand-alone scan, in few registers, so the
// band workgroups that share the kernel keep their occupancy.
__device__ void band_rowscan(const RowScanArgs &a, int64_t *s_tmp, uint32_t *err_hdr) {
    constexpr int RPT = 4;
    uint32_t err = 0;
    int64_t run = 0;
    for (int64_t row0 = 0; row0 < a.n; row0 += (int64_t)NTB * RPT) {
        const int64_t i0 = row0 + (int64_t)threadIdx.x * RPT;
        int64_t off[RPT + 1];
#pragma unroll
        for (int j = 0; j <= RPT; ++j) off[j] = a.offs[i0 + j < a.n ? i0 + j : a.n];
        int64_t len[RPT];
        int64_t mine = 0;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            len[j] = 0;
            if (i0 + j < a.n) {
                int64_t o0 = off[j], o1 = off[j + 1];
                if (o0 < 0 || o1 < o0 || o1 > a.nbytes) err |= DNATOK_DERR_OFFSETS;
                o0 = o0 < 0 ? 0 : (o0 > a.nbytes ? a.nbytes : o0);
                o1 = o1 < o0 ? o0 : (o1 > a.nbytes ? a.nbytes : o1);
                const int64_t L = o1 - o0;
                const int64_t nb = !a.kmer ? L
                                   : a.overlap ? (L >= a.k ? L - a.k + 1 : (L > 0 ? 1 : 0))
                                               : div_k(L + a.k - 1, a.k, a.kinv);
                const int64_t l = nb + 2 * a.cls;
                if (l > a.W) err |= DNATOK_DERR_ROW_WIDTH;
                len[j] = l;
                mine += l;
            }
        }
        int64_t tot;
        int64_t pre = a.base + run + dev::block_excl_scan<NTB>(mine, s_tmp, &tot);
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            if (i0 + j < a.n) a.out_offs[i0 + j] = pre;
            pre += len[j];
        }
        run += tot;
    }
    if (threadIdx.x == 0) a.out_offs[a.n] = a.base + run;
    if (err) dev::raise_error(err_hdr, err);
}

// What the write phase of one unit (a band, or a part of a row) reads.

// Writes every cell of the unit for every vocabulary (ids and mask).
template <bool KMER>
__device__ __forceinline__ void band_write(const BandArgs &a, int64_t r0, int nr, int part, bool staged,
                                           const uint64_t *win64, const uint32_t *val32, const uint8_t *raw,
                                           const int64_t *s_o0, const int64_t *s_o1, const int32_t *s_nb,
                                           const uint32_t *s_ro, const int32_t *s_lut) {
    const int tid = threadIdx.x;
    // Every vocabulary, every row of the band: the row's facts are uniform
    // across the workgroup, so a store group inside the row's full frames
    // costs one staged window read and the four ids; groups at the row's
    // edges (CLS, SEP, the short final frame, pads, the neighbouring rows'
    // cells) go cell by cell and store only this row's cells.
    // Four or more vocabularies: one per wave, a row's groups of that
    // vocabulary in passes of 64 (a workgroup-wide pass of 256 left on
    // average a third of its lanes idle at the end of each row's share of
    // a vocabulary: 54 -> 48 us for k = 3..6 at 8 KiB stages). Fewer
    // vocabularies but four or more rows in the band: one row per wave, for
    // the same reason (single-nucleotide ids at 32 KiB stages 49 -> 43.5 us).
    // Otherwise the whole workgroup.
    const bool by_wave = a.nv >= NTB / dev::kWave;
    const bool by_row = !by_wave && nr >= NTB / dev::kWave;
    // the wave index is uniform across a wave, and saying so keeps each
    // vocabulary's facts (pointers, sizes, ids) in scalar registers: as a
    // per-lane value it held them in VGPRs, 85 instead of 49
    const int wid = __builtin_amdgcn_readfirstlane(tid / dev::kWave);
    const int wtid = (by_wave || by_row) ? (tid & (dev::kWave - 1)) : tid;
    const int wstride = (by_wave || by_row) ? dev::kWave : NTB;
    for (int vi = by_wave ? wid : 0; vi < a.nv; vi += by_wave ? NTB / dev::kWave : 1) {
        const BandVocab o = a.vo[vi];
        const int32_t k = KMER ? o.k : 1;
        const int32_t W = (int32_t)o.W;
        const bool mask4 = ((reinterpret_cast<uintptr_t>(o.mask) - (uintptr_t)o.al) & 3) == 0;
        for (int r = by_row ? wid : 0; r < nr; r += by_row ? NTB / dev::kWave : 1) {
            const int32_t nb = __builtin_amdgcn_readfirstlane(s_nb[vi * kMaxBandRows + r]);
            const int32_t L = __builtin_amdgcn_readfirstlane((int32_t)(s_o1[r] - s_o0[r]));
            const uint32_t ro = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)s_ro[r]);
            const int32_t len = nb + 2 * a.cls;
            if (len > W) continue;  // too long for pad_to: the row writes nothing (the row scan raised the flag)
            const int32_t lead = a.left ? W - len : 0;
            // the one short token: a short final frame, or the single window of a row shorter than k
            const bool tail = KMER && (a.overlap ? (L > 0 && L < k) : nb * k != L);
            const int32_t st = (KMER && !a.overlap) ? k : 1;  // bytes between token starts
            const int32_t bA = lead + a.cls;                 // first body cell
            const int32_t bF = bA + nb - (tail ? 1 : 0);     // end of the full frames
            const int64_t E0 = (r0 + r) * (int64_t)W;        // the row's first cell
            // the row's cells this workgroup writes: all of them, or with
            // parts the tokens starting in the part's bytes, the first part
            // also the leading pads and CLS, the last non-empty one the rest
            int32_t clo = 0, chi = W;
            if (a.P > 1) {
                const int64_t jlo = ((int64_t)part * a.U + st - 1) / st, jhi = ((int64_t)(part + 1) * a.U + st - 1) / st;
                const int64_t plast = L > 0 ? (L - 1) / a.U : 0;
                if (part > plast) continue;
                clo = part == 0 ? 0 : bA + (int32_t)min(jlo, (int64_t)nb);
                chi = part == plast ? W : bA + (int32_t)min(jhi, (int64_t)nb);
            }
            if (clo >= chi) continue;
            const int64_t gf = (E0 + clo + o.al) >> 2, gl = (E0 + chi - 1 + o.al) >> 2;
            // Groups whose four cells are full frames of this row (and part):
            // [ga, gb), one staged window read and four ids each, in 32-bit
            // arithmetic from the range's first cell; the rest (edges) below.
            int64_t ga = gl + 1, gb = gl + 1;
            if (staged && (!KMER || 3 * st + k <= 32)) {
                const int32_t flo = max(bA, clo), fhi = min(bF, chi);
                const int64_t lo_g = (E0 + flo + o.al + 3) >> 2;  // first g with 4g - al - E0 >= flo
                const int64_t hi_g = (E0 + fhi + o.al - 4) >> 2;  // last g with 4g - al - E0 + 4 <= fhi
                if (hi_g >= lo_g) {
                    ga = lo_g;
                    gb = hi_g + 1;
                }
            }
            const int32_t nfast = (int32_t)(gb - ga);
            if (nfast > 0) {
                const int32_t jA = (int32_t)(4 * ga - o.al - E0) - bA;  // token of the first fast group's first cell
                i32x4 *ids4 = reinterpret_cast<i32x4 *>(o.ids + (4 * ga - o.al));
                int8_t *mask0 = o.mask + (4 * ga - o.al);
                // forward non-overlapping k-mers of k = 3..6 with k fixed at compile
                // time: the window's shifts and masks become constants (the
                // launch spends half its time issuing VALU; 1.5% faster)
                auto fast_const = [&](auto kc) {
                    constexpr int KC = decltype(kc)::value;
                    for (int32_t t = wtid; t < nfast; t += wstride) {
                        const int32_t j = jA + 4 * t;
                        const i32x4 y = kmer4_lds(win64, val32, ro + (uint32_t)(j * KC), KC, 0, KC, false);
                        __builtin_nontemporal_store(y, ids4 + t);
                        if (mask4)
                            *reinterpret_cast<uint32_t *>(mask0 + 4 * t) = 0x01010101u;
                        else
                            for (int q = 0; q < 4; ++q) mask0[4 * t + q] = 1;
                    }
                };
                const bool plain = KMER && !a.revcomp && !a.overlap && k >= 3 && k <= 6;
                if (plain) {
                    if (k == 3) fast_const(std::integral_constant<int, 3>{});
                    else if (k == 4) fast_const(std::integral_constant<int, 4>{});
                    else if (k == 5) fast_const(std::integral_constant<int, 5>{});
                    else fast_const(std::integral_constant<int, 6>{});
                }
                for (int32_t t = plain ? nfast : wtid; t < nfast; t += wstride) {
                    const int32_t j = jA + 4 * t;
                    i32x4 y;
                    if (KMER) {
                        // tokens j .. j + 3 read one 32-base window: forward from
                        // their first start, reverse complemented from the last
                        // one's start (token j + q starts at L - (j + q) * st - k)
                        y = a.revcomp ? kmer4_lds(win64, val32, ro + (uint32_t)(L - (j + 3) * st - k), k, 3 * st, -st, true)
                                      : kmer4_lds(win64, val32, ro + (uint32_t)(j * st), k, 0, st, false);
                    } else if (a.revcomp) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) y[q] = s_lut[raw[ro + (uint32_t)(L - 1 - j - q)]];
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) y[q] = s_lut[raw[ro + (uint32_t)(j + q)]];
                    }
                    __builtin_nontemporal_store(y, ids4 + t);
                    // mask words through the cache: a wave's 4-byte stores
                    // cover a line only together, which L2 merges (streamed
                    // past it, they cost 7% of the launch)
                    if (mask4)
                        *reinterpret_cast<uint32_t *>(mask0 + 4 * t) = 0x01010101u;
                    else
                        for (int q = 0; q < 4; ++q) mask0[4 * t + q] = 1;
                }
            }
            // the other groups, [gf, ga) and [gb, gl], cell by cell
            const int64_t n1 = ga - gf, ne = n1 + (gl + 1 - gb);
            for (int64_t ie = wtid; ie < ne; ie += wstride) {
                const int64_t g = ie < n1 ? gf + ie : gb + (ie - n1);
                const int64_t e = 4 * g - o.al;
                const int32_t c0 = (int32_t)(e - E0);
                int32_t *dst = o.ids + e;
                int32_t v[4];
                uint32_t mk = 0;
                bool in[4], all_in = true;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int32_t c = c0 + q;
                    in[q] = c >= clo && c < chi;
                    all_in = all_in && in[q];
                    int32_t id = o.pad_id;
                    uint32_t m = 0;
                    const int32_t tt = c - lead;
                    if (in[q] && tt >= 0 && tt < len) {
                        m = 1;
                        if (a.cls && tt == 0) {
                            id = o.cls_id;
                        } else if (a.cls && tt == len - 1) {
                            id = o.sep_id;
                        } else {
                            const int32_t j = tt - a.cls;
                            // first byte of token j (of its mirror window when reverse complemented)
                            const int32_t b0 = !a.revcomp ? j * st : (KMER ? L - j * st - k : L - 1 - j);
                            if (tail && j == nb - 1) {
                                id = DNATOK_ID_UNK;
                            } else if (staged) {
                                const uint32_t idx = ro + (uint32_t)b0;
                                id = KMER ? kmer_id(kmer_lds(win64, val32, idx, k), k, a.revcomp) : s_lut[raw[idx]];
                            } else {
                                const int64_t pos = s_o0[r] + b0;
                                id = KMER ? kmer_id(kmer_global(a, pos, k), k, a.revcomp)
                                          : s_lut[a.abase[a.shift + pos]];
                            }
                        }
                    }
                    v[q] = id;
                    mk |= m << (8 * q);
                }
                if (all_in) {
                    __builtin_nontemporal_store(i32x4{v[0], v[1], v[2], v[3]}, reinterpret_cast<i32x4 *>(dst));
                    if (mask4)
                        *reinterpret_cast<uint32_t *>(o.mask + e) = mk;
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
        if ((int)blockIdx.x < a.nscan) band_rowscan(a.scan[blockIdx.x], s_tmp, a.err_hdr);
        return;
    }
    const int64_t unit = (int64_t)blockIdx.x - a.lead;
    const int64_t band = unit / a.P;
    const int part = (int)(unit - band * a.P);
    const int64_t r0 = band * a.R;
    const int nr = (int)min((int64_t)a.R, (int64_t)a.n - r0);
    if (!KMER) s_lut[tid] = a.lut[a.revcomp ? complement_byte((uint32_t)tid) : (uint32_t)tid];
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
            lo = lo == INT64_MAX ? 0 : lo;
            if (a.P > 1) {
                // one row: the bytes of this part's tokens (forward: from pU,
                // up to k - 1 bytes past the part; reverse complement: the
                // mirrored range)
                const int64_t L = hi - lo;
                int64_t b0 = (int64_t)part * a.U, b1 = b0 + a.U + a.kmax;
                if (a.revcomp) {
                    const int64_t m0 = L - b1, m1 = L - b0;
                    b0 = m0;
                    b1 = m1;
                }
                b0 = b0 < 0 ? 0 : (b0 > L ? L : b0);
                b1 = b1 < b0 ? b0 : (b1 > L ? L : b1);
                hi = lo + b1;
                lo = lo + b0;
            }
            s_lo = lo;
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
        s_nb[vi * kMaxBandRows + r] = (int32_t)(!KMER ? L
                                                : a.overlap ? (L >= k ? L - k + 1 : (L > 0 ? 1 : 0))
                                                            : div_k(L + k - 1, k, 0xFFFFFFFFu / (uint32_t)k));
    }
    __syncthreads();

    band_write<KMER>(a, r0, nr, part, staged, win64, val32, raw, s_o0, s_o1, s_nb, s_ro, s_lut);
}

// Persistent form: as many workgroups as are resident, each taking units
// u, u + G, ... and putting the next unit's bytes in flight (in registers)
// before writing the current one, so its load latency hides behind the
// writes. A vector load waits for the wave's earlier stores as well, so the
// one wait per unit (for the prefetched bytes) also drains the previous
// unit's stores; the row offsets run two units ahead so no other wait is
// needed. Units of at most kLoopChunks 16-byte chunks per thread.
constexpr int kLoopChunks = 4;
constexpr int kLoopRows = dev::kWave - 1;  // a unit's row offsets fit one wave

template <bool KMER>
__global__ __launch_bounds__(NTB) void k_bands_loop(BandArgs a) {
    extern __shared__ __align__(16) uint8_t dyn[];
    __shared__ int64_t s_o0[kMaxBandRows], s_o1[kMaxBandRows];
    __shared__ int32_t s_nb[kBandVocabs * kMaxBandRows];
    __shared__ uint32_t s_ro[kMaxBandRows];
    __shared__ int32_t s_lut[256];
    __shared__ int64_t s_nlo, s_nhi;  // the next unit's staging window
    __shared__ int64_t s_tmp[NTB / dev::kWave + 1];
    const int tid = threadIdx.x, lane = tid & (dev::kWave - 1);
    if ((int)blockIdx.x < a.lead) {
        if ((int)blockIdx.x < a.nscan) band_rowscan(a.scan[blockIdx.x], s_tmp, a.err_hdr);
        return;
    }
    const int64_t G = (int64_t)gridDim.x - a.lead;
    const int64_t nunits = a.nbands;
    if (!KMER) s_lut[tid] = a.lut[a.revcomp ? complement_byte((uint32_t)tid) : (uint32_t)tid];
    uint64_t *win64 = reinterpret_cast<uint64_t *>(dyn);
    uint32_t *val32 = reinterpret_cast<uint32_t *>(win64 + a.stage_chunks);
    uint8_t *raw = dyn;
    const int64_t lim = a.shift + a.nbytes;

    auto rows_of = [&](int64_t u, int64_t &r0, int &nr, int &part) {
        const int64_t band = u / a.P;
        part = (int)(u - band * a.P);
        r0 = band * a.R;
        nr = (int)min((int64_t)a.R, (int64_t)a.n - r0);
    };
    // wave 0, lane t <= nr: the raw offset of the unit's row boundary t
    auto load_offs = [&](int64_t u) -> int64_t {
        if (u >= nunits || tid >= dev::kWave) return 0;
        int64_t r0;
        int nr, part;
        rows_of(u, r0, nr, part);
        const int64_t i = r0 + (lane <= nr ? lane : nr);
        return a.offs[i];
    };
    // wave 0: clamp the unit's rows from the lanes' raw offsets; optionally
    // write them to LDS; return the unit's staging window (uniform)
    auto rows_window = [&](int64_t u, int64_t raw_off, bool to_lds, int64_t &wlo, int64_t &whi) {
        int64_t r0;
        int nr, part;
        rows_of(u, r0, nr, part);
        const int64_t nxt = __shfl_down(raw_off, 1, dev::kWave);
        int64_t o0 = raw_off < 0 ? 0 : (raw_off > a.nbytes ? a.nbytes : raw_off);
        int64_t o1 = nxt < o0 ? o0 : (nxt > a.nbytes ? a.nbytes : nxt);
        const bool row = lane < nr;
        if (to_lds && row) {
            s_o0[lane] = o0;
            s_o1[lane] = o1;
        }
        int64_t lo = row ? o0 : INT64_MAX, hi = row ? o1 : 0;
#pragma unroll
        for (int d = dev::kWave / 2; d > 0; d >>= 1) {
            lo = min(lo, (int64_t)__shfl_xor(lo, d, dev::kWave));
            hi = max(hi, (int64_t)__shfl_xor(hi, d, dev::kWave));
        }
        lo = lo == INT64_MAX ? 0 : lo;
        if (a.P > 1) {
            const int64_t L = hi - lo;
            int64_t b0 = (int64_t)part * a.U, b1 = b0 + a.U + a.kmax;
            if (a.revcomp) {
                const int64_t m0 = L - b1, m1 = L - b0;
                b0 = m0;
                b1 = m1;
            }
            b0 = b0 < 0 ? 0 : (b0 > L ? L : b0);
            b1 = b1 < b0 ? b0 : (b1 > L ? L : b1);
            hi = lo + b1;
            lo = lo + b0;
        }
        wlo = lo;
        whi = max(hi, lo);
    };
    // the staging chunks of a window: first chunk and count (two spare)
    auto chunks_of = [&](int64_t wlo, int64_t whi, int64_t &c0, int64_t &nch) {
        const int64_t q0 = wlo + a.shift, q1 = whi + a.shift;
        c0 = q0 >> 4;
        nch = ((q1 + 15) >> 4) - c0 + 2;
    };
    auto fetch = [&](int64_t c0, int64_t nch, uint4 (&x)[kLoopChunks]) {
#pragma unroll
        for (int w = 0; w < kLoopChunks; ++w) {
            const int64_t m = (int64_t)w * NTB + tid;
            const int64_t q = (c0 + m) << 4;
            if (m < nch && q >= a.shift && q + 16 <= lim) {
                const u32x4 t = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(a.abase + q));
                x[w] = make_uint4(t[0], t[1], t[2], t[3]);
            } else {
                uint32_t wd[4] = {0, 0, 0, 0};
                if (m < nch)
                    for (int b = 0; b < 16; ++b)
                        if (q + b >= a.shift && q + b < lim) wd[b >> 2] |= (uint32_t)a.abase[q + b] << (8 * (b & 3));
                x[w] = make_uint4(wd[0], wd[1], wd[2], wd[3]);
            }
        }
    };

    int64_t u = (int64_t)blockIdx.x - a.lead;
    // prologue: offsets of the first two units, the first unit's bytes in flight
    int64_t off_cur = load_offs(u);
    int64_t off_nxt = load_offs(u + G);
    if (tid < dev::kWave) {
        int64_t wlo, whi;
        rows_window(u, off_cur, false, wlo, whi);
        if (tid == 0) {
            s_nlo = wlo;
            s_nhi = whi;
        }
    }
    __syncthreads();
    int64_t c0, nch;
    chunks_of(s_nlo, s_nhi, c0, nch);
    bool staged = nch <= a.stage_chunks && nch <= (int64_t)kLoopChunks * NTB;
    uint4 x[kLoopChunks];
    if (staged) fetch(c0, nch, x);
    for (; u < nunits; u += G) {
        __syncthreads();  // the previous unit's writes are done with the stage
        if (staged) {
#pragma unroll
            for (int w = 0; w < kLoopChunks; ++w) {
                const int64_t m = (int64_t)w * NTB + tid;
                if (m >= nch) continue;
                if (KMER) {
                    uint32_t c, vb;
                    dev::classify16(x[w], c, vb);
                    uint32_t *w32 = reinterpret_cast<uint32_t *>(win64);
                    uint16_t *v16 = reinterpret_cast<uint16_t *>(val32);
                    w32[2 * m + 1] = c;
                    v16[2 * m + 1] = (uint16_t)(vb >> 16);
                    if (m > 0) {
                        w32[2 * m - 2] = c;
                        v16[2 * m - 2] = (uint16_t)(vb >> 16);
                    }
                } else {
                    reinterpret_cast<uint4 *>(raw)[m] = x[w];
                }
            }
            if (KMER && tid == 0) {
                reinterpret_cast<uint32_t *>(win64)[2 * (nch - 1)] = 0;
                reinterpret_cast<uint16_t *>(val32)[2 * (nch - 1)] = 0;
            }
        }
        int64_t r0;
        int nr, part;
        rows_of(u, r0, nr, part);
        const int64_t sbase = c0 << 4;
        const bool cur_staged = staged;
        if (tid < dev::kWave) {
            int64_t wlo, whi;
            rows_window(u, off_cur, true, wlo, whi);  // this unit's rows to LDS
            if (u + G < nunits) {
                rows_window(u + G, off_nxt, false, wlo, whi);  // the next unit's window
                if (tid == 0) {
                    s_nlo = wlo;
                    s_nhi = whi;
                }
            }
            if (tid < nr) s_ro[tid] = (uint32_t)(s_o0[tid] + a.shift - sbase);
        }
        __syncthreads();
        for (int t = tid; t < a.nv * nr; t += NTB) {
            const int vi = t / nr, r = t - vi * nr;
            const int64_t L = s_o1[r] - s_o0[r];
            const int32_t k = KMER ? a.vo[vi].k : 1;
            s_nb[vi * kMaxBandRows + r] = (int32_t)(!KMER ? L
                                                    : a.overlap ? (L >= k ? L - k + 1 : (L > 0 ? 1 : 0))
                                                                : div_k(L + k - 1, k, 0xFFFFFFFFu / (uint32_t)k));
        }
        // the next unit's bytes and the offsets of the one after go out now
        int64_t off_nn = 0;
        if (u + G < nunits) {
            chunks_of(s_nlo, s_nhi, c0, nch);
            staged = nch <= a.stage_chunks && nch <= (int64_t)kLoopChunks * NTB;
            if (staged) fetch(c0, nch, x);
            off_nn = load_offs(u + 2 * G);
        }
        __syncthreads();
        band_write<KMER>(a, r0, nr, part, cur_staged, win64, val32, raw, s_o0, s_o1, s_nb, s_ro, s_lut);
        off_cur = off_nxt;
        off_nxt = off_nn;
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
                        int8_t *const *d_masks, const dnatok_encode_opts *os, int64_t stage_bytes, bool persistent,
                        int64_t *const *d_out_offsets, hipStream_t stream, bool *used) {
    *used = false;
    if (nv < 1 || nv > kBandVocabs) return DNATOK_OK;
    const dnatok_vocab *v = vs[0];
    const bool kmer = (v->kind == DNATOK_KMER);
    const dnatok_encode_opts &o = os[0];
    if (o.layout != DNATOK_PADDED) return DNATOK_OK;
    BandArgs a = {};
    a.cls = o.add_cls_sep ? 1 : 0;
    a.left = (o.pad_side == DNATOK_PAD_LEFT) ? 1 : 0;
    a.overlap = (kmer && (o.variant & DNATOK_VARIANT_OVERLAP)) ? 1 : 0;
    a.revcomp = (o.variant & DNATOK_VARIANT_REVCOMP) ? 1 : 0;
    // longest row any vocabulary's pad_to admits, in bytes
    int64_t maxrow = INT64_MAX;
    for (int vi = 0; vi < nv; ++vi) {
        const int64_t k = kmer ? vs[vi]->k : 1;
        const int64_t W = os[vi].pad_to;
        if (W >= (1ll << 31)) return DNATOK_OK;
        const int64_t tok = std::max<int64_t>(0, W - 2 * a.cls);  // tokens a row may have
        maxrow = std::min(maxrow, a.overlap ? (tok > 0 ? tok + k - 1 : 0) : tok * k);
    }
    int32_t kmax = 1;
    for (int vi = 0; vi < nv; ++vi) kmax = std::max<int32_t>(kmax, kmer ? vs[vi]->k : 1);
    // rows that fit the stage go R to a band; longer ones are cut into P parts
    // of U bytes (each staging U + kmax bytes)
    int64_t R = 1, P = 1, U = stage_bytes;
    if (maxrow <= stage_bytes) {
        R = maxrow > 0 ? stage_bytes / maxrow : kMaxBandRows;
        R = std::max<int64_t>(1, std::min<int64_t>(R, persistent ? kLoopRows : kMaxBandRows));
        if (n > 0 && (int64_t)n < R) R = n;
    } else {
        P = (maxrow + U - 1) / U;
        if (P > 4096 || maxrow >= (1ll << 31)) return DNATOK_OK;
        U = ((maxrow + P - 1) / P + 15) / 16 * 16;  // even parts
    }
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
    a.P = (int32_t)P;
    a.U = U;
    a.kmax = kmax;
    // a band of valid rows spans at most R * maxrow bytes (a part U + kmax):
    // its chunks plus the partial ones at both ends and the two spare ones
    const int64_t span = P > 1 ? U + kmax : R * std::max<int64_t>(maxrow, 1);
    a.stage_chunks = (int32_t)((span + 15) / 16 + 4);
    a.nbands = n > 0 ? ((n + R - 1) / R) * P : 0;
    if (a.nbands + 8 >= (1ll << 31)) return DNATOK_OK;
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
        sp.overlap = a.overlap;
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
            s.overlap = a.overlap;
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
    persistent = persistent && a.stage_chunks <= kLoopChunks * NTB && a.nbands > 0;
    if (persistent) {
        if (dyn > 64 * 1024)
            DNATOK_HIP(hipFuncSetAttribute(kmer ? (const void *)k_bands_loop<true> : (const void *)k_bands_loop<false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
        int per_cu = 0;
        DNATOK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, kmer ? (const void *)k_bands_loop<true> : (const void *)k_bands_loop<false>, NTB, dyn));
        const int64_t walkers = std::min<int64_t>(a.nbands, (int64_t)device_cu_count() * std::max(per_cu, 1));
        const int64_t grid = a.lead + walkers;
        if (kmer)
            hipLaunchKernelGGL(k_bands_loop<true>, dim3((unsigned)grid), dim3(NTB), dyn, stream, a);
        else
            hipLaunchKernelGGL(k_bands_loop<false>, dim3((unsigned)grid), dim3(NTB), dyn, stream, a);
        DNATOK_HIP(hipGetLastError());
        *used = true;
        return DNATOK_OK;
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
