// Row scan of the closed-form token counts (shared by the tile kernel, the
// cell kernel and the stand-alone scan launch): each row's length is L, its
// number of k-frames ceil(L / k), or its number of stride-1 windows, plus
// the specials; out_offsets is their exclusive scan. Offsets are validated
// and clamped here, so every kernel that places cells from them agrees.
#pragma once

#include "common.hpp"
#include "device.hpp"

namespace dnatok {

namespace {

constexpr int kScanNT = 256;                                 // block size of every launch that scans
constexpr int kRowsPerThread = 16;                           // rows per thread per pass
constexpr int64_t kUnitRows = (int64_t)kScanNT * kRowsPerThread;

// x / k for k >= 1 with kinv = floor((2^32 - 1) / k): the high product is
// floor(x / k) or one less (x < 2^32), and one step corrects it. Quotients
// of 2^31 or more take the plain division.
__device__ __forceinline__ int64_t div_k(int64_t x, int32_t k, uint32_t kinv) {
    if (x < 0x7FFFFFFF) {
        const uint32_t ux = (uint32_t)x;
        uint32_t q = __umulhi(ux, kinv);
        if (ux - q * (uint32_t)k >= (uint32_t)k) ++q;
        return (int64_t)q;
    }
    return x / k;
}

struct RowScanArgs {
    const int64_t *offs;
    int32_t n;
    int64_t nbytes;
    int64_t *out_offs;
    int32_t k;
    uint32_t kinv;  // floor((2^32 - 1) / k)
    int32_t kmer;
    int32_t overlap;  // k-mer windows of stride 1: L - k + 1 (one for 0 < L < k)
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
    // all of this thread's offsets first, from indices clamped to the batch,
    // so the loads go out together instead of one per row behind its test
    int64_t off[kRowsPerThread + 1];
#pragma unroll
    for (int j = 0; j <= kRowsPerThread; ++j) {
        const int64_t i = i0 + j;
        off[j] = a.offs[i < a.n ? i : a.n];
    }
    int64_t len[kRowsPerThread];
    int64_t mine = 0;
#pragma unroll
    for (int j = 0; j < kRowsPerThread; ++j) {
        const int64_t i = i0 + j;
        len[j] = 0;
        if (i < a.n) {
            int64_t o0 = off[j], o1 = off[j + 1];
            if (o0 < 0 || o1 < o0 || o1 > a.nbytes) err |= DNATOK_DERR_OFFSETS;
            o0 = o0 < 0 ? 0 : (o0 > a.nbytes ? a.nbytes : o0);
            o1 = o1 < o0 ? o0 : (o1 > a.nbytes ? a.nbytes : o1);
            const int64_t L = o1 - o0;
            int64_t nb = L;
            if (a.kmer) nb = a.overlap ? (L >= a.k ? L - a.k + 1 : (L > 0 ? 1 : 0)) : div_k(L + a.k - 1, a.k, a.kinv);
            len[j] = nb + 2 * a.cls;
            if (a.padded && len[j] > a.W) err |= DNATOK_DERR_ROW_WIDTH;
        }
        mine += len[j];
    }
    int64_t total;
    const int64_t pre = dev::block_excl_scan<kScanNT>(mine, s_tmp, &total);
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
[[maybe_unused]] __device__ void rowscan_single_block(const RowScanArgs &a, int64_t *s_tmp, uint32_t *err_hdr) {
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

}  // namespace

}  // namespace dnatok
