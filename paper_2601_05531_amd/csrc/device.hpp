// Device-side building blocks: wave64 scans, block scans, and the one-pass
// (decoupled look-back) tile prefix used by the encode and decode kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/dnatok.h"

namespace dnatok {
namespace dev {

constexpr int kWave = 64;

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_relaxed32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed32(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Inclusive scan across the 64 lanes of a wave.
__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int64_t u = __shfl_up(v, d, kWave);
        if (lane >= d) v += u;
    }
    return v;
}

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Cross-lane moves through DPP (data-parallel primitives of the VALU, no LDS
// round trip). Lanes whose source is outside the pattern, or whose row is
// masked off, return `old`.
template <int CTRL, int ROW_MASK = 0xF, int BANK_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, BANK_MASK, false);
}
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShr1 = 0x138;

// Inclusive sum over the 64 lanes: shifts of 1, 2, 4, 8 inside each row of
// 16 lanes, then the last lane of row 0 / 2 into rows 1 / 3, then lane 31
// into rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_sum_u32(uint32_t v) {
    v += dpp_u32<kDppRowShr1>(0, v);
    v += dpp_u32<kDppRowShr2>(0, v);
    v += dpp_u32<kDppRowShr4>(0, v);
    v += dpp_u32<kDppRowShr8>(0, v);
    v += dpp_u32<kDppRowBcast15, 0xA>(0, v);
    v += dpp_u32<kDppRowBcast31, 0xC>(0, v);
    return v;
}

// Minimum over the 64 lanes, returned to every lane (a prefix minimum
// whose last lane is read back as a scalar).
__device__ __forceinline__ uint32_t wave_min_all_u32(uint32_t v) {
    v = min(v, dpp_u32<kDppRowShr1>(~0u, v));
    v = min(v, dpp_u32<kDppRowShr2>(~0u, v));
    v = min(v, dpp_u32<kDppRowShr4>(~0u, v));
    v = min(v, dpp_u32<kDppRowShr8>(~0u, v));
    v = min(v, dpp_u32<kDppRowBcast15, 0xA>(~0u, v));
    v = min(v, dpp_u32<kDppRowBcast31, 0xC>(~0u, v));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Bitwise or over the 64 lanes, returned to every lane.
__device__ __forceinline__ uint32_t wave_or_all_u32(uint32_t v) {
    v |= dpp_u32<kDppRowShr1>(0u, v);
    v |= dpp_u32<kDppRowShr2>(0u, v);
    v |= dpp_u32<kDppRowShr4>(0u, v);
    v |= dpp_u32<kDppRowShr8>(0u, v);
    v |= dpp_u32<kDppRowBcast15, 0xA>(0u, v);
    v |= dpp_u32<kDppRowBcast31, 0xC>(0u, v);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Value of lane - 1 (lane 0 gets `first`).
__device__ __forceinline__ uint32_t wave_from_prev_u32(uint32_t v, uint32_t first) {
    return dpp_u32<kDppWaveShr1>(first, v);
}

// Value of a lane given by a wave-uniform index.
__device__ __forceinline__ uint32_t wave_read_u32(uint32_t v, uint32_t lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)__builtin_amdgcn_readfirstlane((int)lane));
}

// Block-wide exclusive scan (NT threads, NT a multiple of 64). `tmp` holds
// NT/64 + 1 int64 in LDS. Returns the exclusive prefix; *total gets the sum.
template <int NT>
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *tmp, int64_t *total) {
    constexpr int NW = NT / kWave;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int64_t inc = wave_incl_scan(v);
    if (lane == kWave - 1) tmp[w] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        int64_t t = tmp[i];
        if (i < w) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

template <int NT>
__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t *tmp) {
    constexpr int NW = NT / kWave;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    v = wave_sum(v);
    if (lane == 0) tmp[w] = v;
    __syncthreads();
    int64_t all = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) all += tmp[i];
    __syncthreads();
    return all;
}

// 16 bytes -> 16 two-bit base digits (most significant first) and 16
// validity bits (bit 31 = first byte) for the A/C/G/T/a/c/g/t test. Per 4
// bytes: fold case, read the digit off bits 1-2 (a->0 c->1 g->2 t->3), look
// the canonical letter of that digit up with a byte permute, and compare;
// multiplies gather the 2-bit digits and the validity bits.
__device__ __forceinline__ void classify16(uint4 v, uint32_t &code, uint32_t &valid) {
    const uint32_t x[4] = {v.x, v.y, v.z, v.w};
    code = 0;
    valid = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t f = x[q] | 0x20202020u;  // only A/a map to a (likewise c, g, t)
        const uint32_t d = ((f >> 1) ^ (f >> 2)) & 0x03030303u;
        const uint32_t canon = __builtin_amdgcn_perm(0u, 0x74676361u, d);  // "acgt"[d] per byte
        const uint32_t z = f ^ canon;
        const uint32_t bad = (((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z) & 0x80808080u;  // byte != letter
        code |= ((d * 0x40100401u) >> 24) << (24 - 8 * q);
        valid |= ((((bad ^ 0x80808080u) >> 7) * 0x80402010u) >> 28) << (28 - 4 * q);
    }
}

// First index in [lo, hi) where the monotone predicate (false...true) holds,
// or hi, found by one wave: 64 probes per round, so 2 rounds cover 4096
// candidates and 3 rounds 262144. All 64 lanes must call it.
template <class Pred>
__device__ __forceinline__ int64_t wave_lower_bound(int64_t lo, int64_t hi, Pred pred) {
    const int lane = threadIdx.x & (kWave - 1);
    while (hi > lo) {
        const int64_t span = hi - lo;
        const int64_t stride = (span + kWave - 1) / kWave;
        const int64_t q = lo + (int64_t)lane * stride;
        const bool p = (q < hi) ? pred(q) : true;
        const uint64_t b = __ballot(p);
        const int f = b ? __builtin_ctzll(b) : kWave;
        const int64_t nhi = lo + (int64_t)f * stride;
        const int64_t nlo = (f == 0) ? lo : lo + (int64_t)(f - 1) * stride + 1;
        hi = nhi < hi ? nhi : hi;
        lo = nlo;
        if (stride == 1) lo = hi;
    }
    return hi;
}

// Tile status word: 2-bit flag in the top bits, 62-bit value below.
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagInc = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;

// Publish this tile's aggregate (single lane) so later tiles can start
// summing it before this tile knows its own prefix.
__device__ __forceinline__ void publish_aggregate(uint64_t *status, int64_t tile, int64_t agg) {
    st_relaxed(status + tile, (tile == 0 ? kFlagInc : kFlagAgg) | (uint64_t)agg);
}

// Most polls of a predecessor's status word before the look-back gives up.
// Every predecessor is held by a block that is already running (tiles go
// out in ticket order, or follow the workgroup index, which the XCDs
// dispatch in order) and publishes within microseconds; a million polls
// (each one a global load and a short sleep) is about a second, so reaching
// the cap means the protocol was broken (e.g. two launches sharing one
// workspace at once), never a slow peer.
constexpr uint32_t kLookbackMaxPolls = 1u << 20;

__device__ __forceinline__ void raise_error(uint32_t *hdr, uint32_t flag) { atomicOr(hdr + 3, flag); }

// Exclusive prefix of all tiles before `tile`, computed by one full wave
// (all 64 lanes call it): each round reads the 64 nearest unread
// predecessors at once, sums back to the closest one that already knows its
// inclusive prefix, and stops there; otherwise it adds all 64 aggregates and
// moves 64 tiles further back. Tile indices below 0 read as an inclusive
// prefix of 0. Afterwards lane 0 publishes this tile's inclusive prefix.
// Tiles are handed out in ticket order (or follow the workgroup index), so
// every predecessor is held by a block that started earlier and never waits
// on a later tile: the wait ends.
// Should a predecessor stay unpublished for kLookbackMaxPolls polls, the
// wave raises DNATOK_DERR_INTERNAL in hdr, counts what it has, and still
// publishes, so no later tile waits on it and the launch drains.
__device__ __forceinline__ int64_t wave_lookback(uint64_t *status, int64_t tile, int64_t agg, uint32_t *hdr) {
    const int lane = threadIdx.x & (kWave - 1);
    int64_t excl = 0;
    int64_t top = tile - 1;
    uint32_t polls = 0;
    while (top >= 0) {
        const int64_t j = top - lane;
        uint64_t w = (j >= 0) ? ld_relaxed(status + j) : kFlagInc;
        const uint64_t f = w & ~kValMask;
        const uint64_t inc_mask = __ballot(f == kFlagInc);
        const uint64_t zero_mask = __ballot(f == 0);
        const int first_inc = inc_mask ? __builtin_ctzll(inc_mask) : kWave;
        // lanes that must be known: 0 .. first_inc (all 64 if no inclusive one)
        const uint64_t need = (first_inc >= kWave - 1) ? ~0ull : ((2ull << first_inc) - 1);
        if ((zero_mask & need) && ++polls < kLookbackMaxPolls) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        if (zero_mask & need) {
            if (lane == 0) raise_error(hdr, DNATOK_DERR_INTERNAL);
            break;
        }
        int64_t v = (lane <= first_inc) ? (int64_t)(w & kValMask) : 0;
        excl += wave_sum(v);
        if (first_inc < kWave) break;
        top -= kWave;
    }
    if (lane == 0) st_relaxed(status + tile, kFlagInc | (uint64_t)(excl + agg));
    return excl;
}

// Workspace header protocol shared by one-pass kernels.
struct TileQueue {
    uint32_t *hdr;       // [ticket, done, parity, err]
    uint64_t *status0;   // parity 0 status words
    uint64_t *status1;   // parity 1 status words
    int64_t clear_n;     // status words of the other parity to zero
};

// Called by thread 0 of every block after its last tile: the last block to
// finish resets the counters and, for kernels that used (and cleared) the
// status words, flips the parity for the next launch. A kernel that only
// takes tickets passes flip = false so the parity stays with the status
// array the next scan expects to be clear.
__device__ __forceinline__ void finish_block(uint32_t *hdr, bool flip = true) {
    uint32_t d = atomicAdd(hdr + 1, 1u);
    if (d == gridDim.x - 1) {
        st_relaxed32(hdr + 0, 0u);
        st_relaxed32(hdr + 1, 0u);
        if (flip) st_relaxed32(hdr + 2, ld_relaxed32(hdr + 2) ^ 1u);
    }
}

}  // namespace dev
}  // namespace dnatok
