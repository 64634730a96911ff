// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dnatok.h"

namespace dnatok {

// ---- errors -----------------------------------------------------------------

int set_error(int code, const char *fmt, ...);
void clear_error();

#define DNATOK_HIP(call)                                                                      \
    do {                                                                                      \
        hipError_t _e = (call);                                                               \
        if (_e != hipSuccess)                                                                 \
            return ::dnatok::set_error(_e == hipErrorOutOfMemory ? DNATOK_ENOMEM : DNATOK_EDEVICE, \
                                       "%s failed: %s", #call, hipGetErrorString(_e));        \
    } while (0)

// ---- allocation -----------------------------------------------------------------
//
// Every device and pinned host allocation of the library goes through these,
// so a test can make one of them fail: with the environment variable
// DNATOK_TEST_FAIL_ALLOC=n (n >= 1), the n-th allocation after the variable
// took that value returns hipErrorOutOfMemory (later ones succeed; counting
// restarts when the value changes; unset, nothing fails).
hipError_t dev_alloc(void **p, size_t bytes);
hipError_t host_alloc(void **p, size_t bytes);

// ---- vocabulary ----------------------------------------------------------------

// Pair -> rank lookup shared by the host (table build) and the device: a
// two-choice cuckoo table of 16-byte buckets, each holding two entries
// (key, rank) with key = left | right << 16 (never 0: left >= 5). A pair is
// in one of its two buckets, so a lookup is two independent 16-byte reads.
__host__ __device__ inline uint32_t bpe_hash1(uint32_t key) {
    uint32_t h = key * 0x9E3779B1u;
    h ^= h >> 15;
    h *= 0x85EBCA77u;
    h ^= h >> 13;
    return h;
}
__host__ __device__ inline uint32_t bpe_hash2(uint32_t key) {
    uint32_t h = (key ^ 0x5BD1E995u) * 0xC2B2AE35u;
    h ^= h >> 16;
    h *= 0x27D4EB2Fu;
    h ^= h >> 15;
    return h;
}
// Bucket of hash h among nbk buckets, and the two buckets of a key.
__host__ __device__ inline uint32_t bpe_bucket(uint32_t h, uint32_t nbk) {
    return (uint32_t)(((uint64_t)h * nbk) >> 32);
}
__host__ __device__ inline void bpe_buckets(uint32_t key, uint32_t nbk, uint32_t *b1, uint32_t *b2) {
    *b1 = bpe_bucket(bpe_hash1(key), nbk);
    uint32_t c = bpe_bucket(bpe_hash2(key), nbk);
    if (c == *b1) c = (*b1 + 1 == nbk) ? 0 : *b1 + 1;
    *b2 = c;
}

constexpr int32_t kBpeMaxMerges = 8192;  // ranks and ids fit 16 bits; tables live in LDS
constexpr uint16_t kNoRank = 0xFFFF;

struct BpeTables {
    int32_t n_merges = 0;
    uint32_t nbk = 0;               // cuckoo buckets
    uint32_t *d_bucket = nullptr;   // [nbk][4]: key0, rank0, key1, rank1 (key 0 = empty)
    uint32_t *d_pair = nullptr;     // [R] left | right << 16
    int32_t *d_tok_len = nullptr;   // decoded length per id, [vocab]
    int64_t *d_tok_off = nullptr;   // offset of each id's bases in d_tok_chars, [vocab]
    uint8_t *d_tok_chars = nullptr;
};

}  // namespace dnatok

struct dnatok_vocab {
    // Scheduling knobs (dnatok_set_tuning / dnatok_autotune); 0 = default.
    // They change how work is tiled, never the ids.
    std::atomic<int32_t> tune_tile{0}, tune_blocks{0}, tune_item{0}, tune_waves{0}, tune_spread{0}, tune_bands{0};
    int32_t kind = 0;
    int32_t k = 1;
    int32_t pad_id = DNATOK_ID_PAD, cls_id = DNATOK_ID_CLS, sep_id = DNATOK_ID_SEP;
    int32_t vocab_size = 0;
    int32_t max_token_bytes = 1;
    int device = 0;
    int32_t *d_lut = nullptr;  // 256 ids (SINGLE table or the user's LUT256)
    std::vector<int32_t> h_merges;
    dnatok::BpeTables bpe;
};

namespace dnatok {

// ---- per-stream device workspace ----------------------------------------------
//
// One-pass scans (decoupled look-back) need, per launch, a ticket counter, a
// done counter, a parity bit and a status word per tile. The header is
// self-resetting: the last block of each launch zeroes the counters and flips
// the parity, and every launch zeroes the status array of the other parity for
// the next one, so no memset is ever enqueued between launches (graph capture
// friendly). One workspace exists per (device, stream).
// Words 8..16 hold the BPE length-class queue counters (counts 4, tickets 4,
// done), zero between launches.
enum HdrSlot { HDR_TICKET = 0, HDR_DONE = 1, HDR_PARITY = 2, HDR_ERR = 3, HDR_WORDS = 4, HDR_BPE_QUEUES = 8 };

struct Workspace {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t *d_hdr = nullptr;     // HDR_WORDS
    uint64_t *d_status = nullptr;  // 2 * cap words (parity 0 then parity 1)
    int64_t cap = 0;               // tiles
    int64_t high_water = 0;        // tiles that may hold non-zero status
    uint8_t *d_scratch = nullptr;  // general scratch for multi-pass kernels (BPE)
    int64_t scratch_bytes = 0;
    bool fixed = false;            // lives in the library's fixed device array: never grows
};

// Workspace for (current device, stream) with room for `tiles` tiles, grown
// (synchronously, outside graph capture) when needed. While a
// FixedWorkspaceScope is open on the calling thread, every launcher gets that
// fixed workspace instead, and a request beyond its size fails with EBUDGET
// (nothing is allocated).
int get_workspace(hipStream_t stream, int64_t tiles, Workspace **out);
// Ensure the workspace scratch holds at least `bytes` bytes (a fixed
// workspace: EBUDGET when it does not).
int ensure_scratch(Workspace *ws, int64_t bytes);
// Routes the calling thread's launches to `ws` until the scope ends.
class FixedWorkspaceScope {
  public:
    explicit FixedWorkspaceScope(Workspace *ws);
    ~FixedWorkspaceScope();
    FixedWorkspaceScope(const FixedWorkspaceScope &) = delete;
    FixedWorkspaceScope &operator=(const FixedWorkspaceScope &) = delete;

  private:
    Workspace *prev_;
};
// Workspace of (current device, stream) if one exists.
Workspace *find_workspace(hipStream_t stream);
// Free the workspace of (current device, stream); the stream must be idle.
void drop_workspace(hipStream_t stream);

int device_cu_count();

// ---- launchers (encode.hip / decode.hip / bpe.hip) ------------------------------

struct EncodeTuning {
    int64_t tile_bytes;  // bytes of input per tile (multiple of 16)
    int blocks_per_cu;   // 0 = as many as occupancy allows
    int spread;          // 0 = static walkers; > 0: ticketed tiles plus this percentage of extra workgroups
    int bands;           // PADDED: 0 = default, 1 = row bands, 2 = tiles, 3 = persistent row bands
};
EncodeTuning encode_tuning(const dnatok_vocab *v, int64_t nbytes);
constexpr int32_t kBpeItemBytesDefault = 8192;  // nominal BPE item length S
constexpr int32_t kBpeItemBytesMin = 1024;

int launch_encode(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                  int32_t n, int32_t *d_ids, int64_t cap, int64_t *d_out_offsets, int8_t *d_mask,
                  const dnatok_encode_opts &o, hipStream_t stream);

// One pass over the input writing the same batch for several vocabularies of
// one kind (SINGLE/LUT256: one; KMER: up to 8, any k), options alike but for
// pad_to and offset_base.
// PADDED encode by row bands (bands.hip). Launches and sets *used when the
// batch suits bands (every row pad_to admits fits stage_bytes), else leaves
// *used false and launches nothing.
int launch_encode_bands(const dnatok_vocab *const *vs, int nv, const uint8_t *d_bytes, int64_t nbytes,
                        const int64_t *d_offsets, int32_t n, int32_t *const *d_ids, const int64_t *caps,
                        int8_t *const *d_masks, const dnatok_encode_opts *os, int64_t stage_bytes, bool persistent,
                        int64_t *const *d_out_offsets, hipStream_t stream, bool *used);

int launch_encode_multi(const dnatok_vocab *const *vs, int nv, const uint8_t *d_bytes, int64_t nbytes,
                        const int64_t *d_offsets, int32_t n, int32_t *const *d_ids, const int64_t *caps,
                        int64_t *const *d_out_offsets, int8_t *const *d_masks, const dnatok_encode_opts *os,
                        hipStream_t stream);

// Row scan of the closed-form token counts: out[i] = base + the sum over
// rows r < i of len_r, len = body + 2 * cls with body = L (kmer = 0),
// ceil(L / k) (frames) or L - k + 1, one for 0 < L < k (overlap). Raises
// DNATOK_DERR_OFFSETS for bad offsets and, PADDED, DNATOK_DERR_ROW_WIDTH
// for a row longer than W.
struct RowScanSpec {
    const int64_t *offs;
    int32_t n;
    int64_t nbytes;
    int64_t *out;
    int32_t k;
    int32_t kmer;
    int32_t overlap;
    int32_t cls;
    int32_t padded;
    int64_t W;
    int64_t base;
};
int launch_rowscan_spec(const RowScanSpec &sp, hipStream_t stream);

// out[i] = sum over rows r < i of ceil(L_r / divisor) + 2 * cls (out[n] = total).
int launch_rowscan(const int64_t *d_offsets, int32_t n, int64_t nbytes, int64_t *d_out, int32_t divisor, int32_t cls,
                   hipStream_t stream);

// One length class of the wave-per-item BPE kernel.
struct BpeClass {
    int waves;       // waves per workgroup
    int32_t lo, hi;  // items with lo < length <= hi
    uint32_t np;     // symbols per wave
    uint32_t lds;    // dynamic LDS bytes per workgroup
};
int bpe_wave_classes(uint32_t table_lds_bytes, int max_waves, BpeClass *out, int max_out);

// Scratch bytes and workspace tiles one BPE encode of (nbytes, n rows) needs
// with nominal item length S.
int64_t bpe_scratch_bytes(int64_t nbytes, int32_t n, int32_t S);
int64_t bpe_workspace_tiles(int64_t nbytes, int32_t n, int32_t S);

int launch_bpe_encode(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                      int32_t n, int32_t *d_ids, int64_t cap, int64_t *d_out_offsets, int8_t *d_mask,
                      const dnatok_encode_opts &o, hipStream_t stream);

// Output-parallel kernels (cellwise.hip): encode variants (reverse
// complement, overlapping k-mers), the fused encode + embedding lookup, and
// the lookup of given ids.
int launch_encode_variant(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                          int32_t n, int32_t *d_ids, int64_t cap, int64_t *d_out_offsets, int8_t *d_mask,
                          const dnatok_encode_opts &o, hipStream_t stream);
int launch_embed(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets, int32_t n,
                 const void *d_table, int64_t n_rows, int64_t row_bytes, void *d_out, int64_t out_rows,
                 int64_t *d_out_offsets, int32_t *d_ids, int8_t *d_mask, const dnatok_encode_opts &o,
                 hipStream_t stream);
// Lookup of given ids: int32 ids (d_ids) or int64 ids (d_ids64, the other NULL).
int launch_embed_ids(const int32_t *d_ids, const int64_t *d_ids64, int64_t n_ids, const void *d_table,
                     int64_t n_rows, int64_t row_bytes, void *d_out, hipStream_t stream);

int launch_decode(const dnatok_vocab *v, const int32_t *d_ids, int64_t n_ids, const int64_t *d_offsets,
                  int32_t n, uint8_t *d_out, int64_t out_capacity, int64_t *d_out_offsets, hipStream_t stream);

}  // namespace dnatok
