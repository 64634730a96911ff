// Exported C-ABI: argument checks, vocabulary construction and per-stream
// workspaces. Device work lives in encode.hip, decode.hip and bpe.hip.
#include <algorithm>
#include <memory>
#include <cstdarg>
#include <cstdlib>
#include <map>
#include <unordered_set>

#include "common.hpp"

namespace dnatok {

namespace {
thread_local std::string g_err = "no error";
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;
std::mutex g_dev_mu;
std::map<int, int> g_cu;
}  // namespace

int set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err = "no error"; }

namespace {
std::mutex g_fail_mu;
std::string g_fail_value;
int64_t g_fail_count = 0;

// Whether the allocation being made is the one DNATOK_TEST_FAIL_ALLOC names.
bool injected_alloc_failure() {
    const char *e = std::getenv("DNATOK_TEST_FAIL_ALLOC");
    std::lock_guard<std::mutex> lk(g_fail_mu);
    if (!e || !*e) {
        g_fail_value.clear();
        g_fail_count = 0;
        return false;
    }
    if (g_fail_value != e) {
        g_fail_value = e;
        g_fail_count = 0;
    }
    const long long n = std::atoll(e);
    return n >= 1 && ++g_fail_count == n;
}
}  // namespace

hipError_t dev_alloc(void **p, size_t bytes) {
    if (injected_alloc_failure()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

hipError_t host_alloc(void **p, size_t bytes) {
    if (injected_alloc_failure()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipHostMalloc(p, bytes, hipHostMallocDefault);
}

int device_cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_cu.find(dev);
    if (it != g_cu.end()) return it->second;
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
    g_cu[dev] = cu;
    return cu;
}

Workspace *find_workspace(hipStream_t stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find({dev, stream});
    return it == g_ws.end() ? nullptr : it->second;
}

void drop_workspace(hipStream_t stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find({dev, stream});
    if (it == g_ws.end()) return;
    Workspace *ws = it->second;
    if (ws) {
        if (ws->d_hdr) (void)hipFree(ws->d_hdr);
        if (ws->d_scratch) (void)hipFree(ws->d_scratch);
        delete ws;
    }
    g_ws.erase(it);
}

static int grow_allowed(hipStream_t stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone)
        return set_error(DNATOK_ESTATE,
                         "the stream's workspace must grow, which cannot happen during graph capture; "
                         "run one uncaptured call of at least this size first");
    return DNATOK_OK;
}

namespace {
thread_local Workspace *t_fixed_ws = nullptr;
}  // namespace

FixedWorkspaceScope::FixedWorkspaceScope(Workspace *ws) : prev_(t_fixed_ws) { t_fixed_ws = ws; }
FixedWorkspaceScope::~FixedWorkspaceScope() { t_fixed_ws = prev_; }

int get_workspace(hipStream_t stream, int64_t tiles, Workspace **out) {
    if (t_fixed_ws) {
        if (tiles > t_fixed_ws->cap)
            return set_error(DNATOK_EBUDGET, "the batch needs %lld scan tiles, the fixed scratch holds %lld",
                             (long long)tiles, (long long)t_fixed_ws->cap);
        *out = t_fixed_ws;
        return DNATOK_OK;
    }
    int dev = 0;
    DNATOK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace *&ws = g_ws[{dev, stream}];
    if (!ws) {
        ws = new Workspace();
        ws->device = dev;
        ws->stream = stream;
    }
    if (tiles > ws->cap) {
        int rc = grow_allowed(stream);
        if (rc) return rc;
        int64_t cap = std::max<int64_t>({tiles, 2 * ws->cap, 4096});
        DNATOK_HIP(hipStreamSynchronize(stream));
        uint32_t err_keep = 0;
        if (ws->d_hdr) {
            DNATOK_HIP(hipMemcpy(&err_keep, ws->d_hdr + HDR_ERR, sizeof(uint32_t), hipMemcpyDeviceToHost));
            DNATOK_HIP(hipFree(ws->d_hdr));
            ws->d_hdr = nullptr;
            ws->d_status = nullptr;
            ws->cap = 0;
        }
        size_t bytes = 256 + (size_t)cap * 2 * sizeof(uint64_t);
        void *p = nullptr;
        DNATOK_HIP(dev_alloc(&p, bytes));
        // zero on the workspace's own stream and wait: a plain hipMemset runs on
        // the null stream, which does not order non-blocking streams
        DNATOK_HIP(hipMemsetAsync(p, 0, bytes, stream));
        DNATOK_HIP(hipStreamSynchronize(stream));
        ws->d_hdr = static_cast<uint32_t *>(p);
        ws->d_status = reinterpret_cast<uint64_t *>(static_cast<uint8_t *>(p) + 256);
        ws->cap = cap;
        ws->high_water = 0;
        if (err_keep) {
            DNATOK_HIP(hipMemcpyAsync(ws->d_hdr + HDR_ERR, &err_keep, sizeof(uint32_t), hipMemcpyHostToDevice, stream));
            DNATOK_HIP(hipStreamSynchronize(stream));
        }
    }
    *out = ws;
    return DNATOK_OK;
}

int ensure_scratch(Workspace *ws, int64_t bytes) {
    if (bytes <= ws->scratch_bytes) return DNATOK_OK;
    if (ws->fixed)
        return set_error(DNATOK_EBUDGET, "the batch needs %lld bytes of scratch, the fixed scratch holds %lld",
                         (long long)bytes, (long long)ws->scratch_bytes);
    int rc = grow_allowed(ws->stream);
    if (rc) return rc;
    int64_t nb = std::max<int64_t>(bytes, 2 * ws->scratch_bytes);
    DNATOK_HIP(hipStreamSynchronize(ws->stream));
    if (ws->d_scratch) DNATOK_HIP(hipFree(ws->d_scratch));
    ws->d_scratch = nullptr;
    ws->scratch_bytes = 0;
    void *p = nullptr;
    DNATOK_HIP(dev_alloc(&p, (size_t)nb));
    ws->d_scratch = static_cast<uint8_t *>(p);
    ws->scratch_bytes = nb;
    return DNATOK_OK;
}

// ---- fixed scratch (dnatok_encode_noalloc) ---------------------------------------
//
// One array per device, allocated with the code object when it loads and held
// until the process ends: a 256-byte header, the status words of both scan
// parities, then the scratch of multi-pass kernels. In host code `scratch`
// names a host-side stand-in, never the device array: every use goes through
// the address hipGetSymbolAddress returns for the current device.
constexpr size_t kFixedScratchBytes = (size_t)32 << 20;
constexpr int64_t kFixedTiles = 16384;  // status words per parity
constexpr size_t kFixedHeadBytes = 256 + (size_t)kFixedTiles * 2 * sizeof(uint64_t);
static_assert(kFixedHeadBytes % 256 == 0, "the scratch area stays 256-byte aligned");
static __device__ __align__(256) uint8_t scratch[kFixedScratchBytes];

namespace {
std::mutex g_fixed_mu;
std::map<int, Workspace *> g_fixed;  // device -> its view of the array

__global__ void k_zero_words(uint64_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}
}  // namespace

// The fixed workspace of the current device. The first call on a device
// resolves the array's device address (with that device current) and clears
// the header and status words with a fill kernel on `stream`, which orders
// the clear before the launches of the call that follows.
static int fixed_workspace(hipStream_t stream, Workspace **out) {
    int dev = 0;
    DNATOK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_fixed_mu);
    auto it = g_fixed.find(dev);
    if (it != g_fixed.end()) {
        *out = it->second;
        return DNATOK_OK;
    }
    uint8_t *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(reinterpret_cast<void **>(&ptr), HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return set_error(DNATOK_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                         hipGetErrorString(e));
    hipLaunchKernelGGL(k_zero_words, dim3(64), dim3(256), 0, stream, reinterpret_cast<uint64_t *>(ptr),
                       (int64_t)(kFixedHeadBytes / sizeof(uint64_t)));
    DNATOK_HIP(hipGetLastError());
    std::unique_ptr<Workspace> ws(new Workspace());
    ws->device = dev;
    ws->stream = nullptr;
    ws->d_hdr = reinterpret_cast<uint32_t *>(ptr);
    ws->d_status = reinterpret_cast<uint64_t *>(ptr + 256);
    ws->cap = kFixedTiles;
    ws->high_water = 0;
    ws->d_scratch = ptr + kFixedHeadBytes;
    ws->scratch_bytes = (int64_t)(kFixedScratchBytes - kFixedHeadBytes);
    ws->fixed = true;
    *out = ws.get();
    g_fixed[dev] = ws.release();
    return DNATOK_OK;
}

// Device flags raised by fixed-scratch calls on the current device (cleared).
static int take_fixed_flags(hipStream_t s, uint32_t *flags) {
    int dev = 0;
    DNATOK_HIP(hipGetDevice(&dev));
    Workspace *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_fixed_mu);
        auto it = g_fixed.find(dev);
        if (it != g_fixed.end()) ws = it->second;
    }
    *flags = 0;
    if (!ws) return DNATOK_OK;
    DNATOK_HIP(hipMemcpy(flags, ws->d_hdr + HDR_ERR, sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (*flags) {
        DNATOK_HIP(hipMemsetAsync(ws->d_hdr + HDR_ERR, 0, sizeof(uint32_t), s));
        DNATOK_HIP(hipStreamSynchronize(s));
    }
    return DNATOK_OK;
}

// ---- vocabulary construction ----------------------------------------------------

static int check_merges(const int32_t *m, int32_t R) {
    std::unordered_set<uint64_t> seen;
    seen.reserve((size_t)R * 2);
    for (int32_t r = 0; r < R; ++r) {
        for (int s = 0; s < 2; ++s) {
            int32_t x = m[2 * r + s];
            bool ok = (x >= 5 && x <= 8) || (x >= 10 && x < 10 + r);
            if (!ok)
                return set_error(DNATOK_EVOCAB,
                                 "merge %d: operand %d is neither a base id (5..8) nor an earlier merge", r, x);
        }
        uint64_t key = ((uint64_t)(uint32_t)m[2 * r] << 32) | (uint32_t)m[2 * r + 1];
        if (!seen.insert(key).second) return set_error(DNATOK_EVOCAB, "merge %d repeats an earlier pair", r);
    }
    return DNATOK_OK;
}

int build_bpe_tables(dnatok_vocab *v);  // bpe.hip
void free_bpe_tables(dnatok_vocab *v);  // bpe.hip

}  // namespace dnatok

using namespace dnatok;

extern "C" {

const char *dnatok_last_error(void) { return g_err.c_str(); }

int32_t dnatok_version(void) { return 100; }

int dnatok_vocab_destroy(dnatok_vocab *v) {
    if (!v) return set_error(DNATOK_EINVAL, "null vocabulary");
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(v->device);
    if (v->d_lut) (void)hipFree(v->d_lut);
    free_bpe_tables(v);
    (void)hipSetDevice(prev);
    delete v;
    return DNATOK_OK;
}

int dnatok_vocab_create(const dnatok_vocab_desc *d, dnatok_vocab **out) {
    if (!d || !out) return set_error(DNATOK_EINVAL, "null argument");
    *out = nullptr;
    std::unique_ptr<dnatok_vocab> v(new dnatok_vocab());
    v->kind = d->kind;
    DNATOK_HIP(hipGetDevice(&v->device));
    int32_t lut[256];
    switch (d->kind) {
    case DNATOK_SINGLE:
    case DNATOK_BPE: {
        for (int b = 0; b < 256; ++b) lut[b] = DNATOK_ID_UNK;
        const char *up = "ACGT", *lo = "acgt";
        for (int j = 0; j < 4; ++j) {
            lut[(uint8_t)up[j]] = 5 + j;
            lut[(uint8_t)lo[j]] = 5 + j;
        }
        lut['N'] = lut['n'] = 9;
        v->vocab_size = 10;
        v->max_token_bytes = 1;
        break;
    }
    case DNATOK_LUT256: {
        if (!d->lut256) return set_error(DNATOK_EVOCAB, "LUT256 needs a 256-entry table");
        int32_t mx = std::max({d->pad_id, d->cls_id, d->sep_id});
        if (d->pad_id < 0 || d->cls_id < 0 || d->sep_id < 0) return set_error(DNATOK_EVOCAB, "negative special id");
        for (int b = 0; b < 256; ++b) {
            if (d->lut256[b] < 0) return set_error(DNATOK_EVOCAB, "negative id for byte %d", b);
            lut[b] = d->lut256[b];
            mx = std::max(mx, lut[b]);
        }
        v->pad_id = d->pad_id;
        v->cls_id = d->cls_id;
        v->sep_id = d->sep_id;
        v->vocab_size = mx + 1;
        v->max_token_bytes = 1;
        break;
    }
    case DNATOK_KMER:
        if (d->k < 1 || d->k > 15) return set_error(DNATOK_EVOCAB, "k must be in 1..15 (got %d)", d->k);
        v->k = d->k;
        v->vocab_size = 5 + (int32_t)(1u << (2 * d->k));
        v->max_token_bytes = d->k;
        for (int b = 0; b < 256; ++b) lut[b] = 0;
        break;
    default:
        return set_error(DNATOK_EVOCAB, "unknown vocabulary kind %d", d->kind);
    }
    if (d->kind == DNATOK_BPE) {
        if (d->n_merges < 0 || (d->n_merges > 0 && !d->merges))
            return set_error(DNATOK_EVOCAB, "BPE needs n_merges >= 0 and a merge table");
        if (d->n_merges > (1 << 24)) return set_error(DNATOK_EVOCAB, "too many merges");
        int rc = check_merges(d->merges, d->n_merges);
        if (rc) return rc;
        v->h_merges.assign(d->merges, d->merges + 2 * (size_t)d->n_merges);
        v->vocab_size = 10 + d->n_merges;
    }
    void *p = nullptr;
    DNATOK_HIP(dev_alloc(&p, 256 * sizeof(int32_t)));
    v->d_lut = static_cast<int32_t *>(p);
    DNATOK_HIP(hipMemcpy(v->d_lut, lut, sizeof(lut), hipMemcpyHostToDevice));
    if (d->kind == DNATOK_BPE) {
        int rc = build_bpe_tables(v.get());
        if (rc) {
            dnatok_vocab_destroy(v.release());
            return rc;
        }
    }
    // copies from pageable memory may still be in flight when hipMemcpy
    // returns; finish them before any stream (blocking or not) reads the tables
    DNATOK_HIP(hipDeviceSynchronize());
    *out = v.release();
    return DNATOK_OK;
}

int dnatok_vocab_info(const dnatok_vocab *v, int32_t *vocab_size, int32_t *max_token_bytes) {
    if (!v) return set_error(DNATOK_EINVAL, "null vocabulary");
    if (vocab_size) *vocab_size = v->vocab_size;
    if (max_token_bytes) *max_token_bytes = v->max_token_bytes;
    return DNATOK_OK;
}

int dnatok_encode_plan(const dnatok_vocab *v, const int64_t *h_offsets, int32_t n, const dnatok_encode_opts *opts,
                       int64_t *total_tokens, int64_t *max_len) {
    if (!v || n < 0 || (!h_offsets && n > 0)) return set_error(DNATOK_EINVAL, "bad argument");
    const int64_t sp = (opts && opts->add_cls_sep) ? 2 : 0;
    const int64_t k = (v->kind == DNATOK_KMER) ? v->k : 1;
    const bool overlap = opts && (opts->variant & DNATOK_VARIANT_OVERLAP) && v->kind == DNATOK_KMER;
    int64_t tot = 0, mx = 0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t L = h_offsets[i + 1] - h_offsets[i];
        if (L < 0) return set_error(DNATOK_EINVAL, "offsets decrease at row %d", i);
        int64_t body = overlap ? (L >= k ? L - k + 1 : (L > 0 ? 1 : 0)) : (L + k - 1) / k;
        int64_t len = body + sp;
        tot += len;
        mx = std::max(mx, len);
    }
    if (total_tokens) *total_tokens = tot;
    if (max_len) *max_len = mx;
    return DNATOK_OK;
}

// Checks an encode's inputs and options (everything but the id and mask
// outputs).
static int check_inputs(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                        int32_t n, int64_t *d_out_offsets, const dnatok_encode_opts &o) {
    if (!v) return set_error(DNATOK_EINVAL, "null vocabulary");
    if (n < 0 || nbytes < 0) return set_error(DNATOK_EINVAL, "negative size");
    if (!d_offsets || !d_out_offsets) return set_error(DNATOK_EINVAL, "offsets and out_offsets are required");
    if (nbytes > 0 && !d_bytes) return set_error(DNATOK_EINVAL, "null bytes");
    if (o.layout != DNATOK_PACKED && o.layout != DNATOK_PADDED) return set_error(DNATOK_EINVAL, "bad layout");
    if (o.pad_side != DNATOK_PAD_RIGHT && o.pad_side != DNATOK_PAD_LEFT) return set_error(DNATOK_EINVAL, "bad pad side");
    if (o.layout == DNATOK_PADDED && o.pad_to <= 0) return set_error(DNATOK_EINVAL, "PADDED needs pad_to > 0");
    if (o.variant & ~(DNATOK_VARIANT_REVCOMP | DNATOK_VARIANT_OVERLAP)) return set_error(DNATOK_EINVAL, "unknown variant flags");
    if (o.variant && v->kind == DNATOK_BPE) return set_error(DNATOK_EVOCAB, "encode variants need SINGLE, LUT256 or KMER");
    if ((o.variant & DNATOK_VARIANT_OVERLAP) && v->kind != DNATOK_KMER)
        return set_error(DNATOK_EINVAL, "overlapping windows need a k-mer vocabulary");
    int dev = 0;
    DNATOK_HIP(hipGetDevice(&dev));
    if (dev != v->device) return set_error(DNATOK_EINVAL, "vocabulary lives on device %d, current is %d", v->device, dev);
    return DNATOK_OK;
}

// Capacity of a PADDED output of `cap` cells against n x pad_to.
static int check_padded_cap(int32_t n, int64_t cap, const dnatok_encode_opts &o, const char *what) {
    if (o.layout == DNATOK_PADDED && (int64_t)n > 0 && o.pad_to > cap / (int64_t)n)
        return set_error(DNATOK_ETOOSMALL, "%s %lld < n * pad_to", what, (long long)cap);
    return DNATOK_OK;
}

// Checks one encode's arguments (everything dnatok_encode checks on the host).
static int check_encode(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                        int32_t n, int32_t *d_ids, int64_t ids_capacity, int64_t *d_out_offsets, int8_t *d_mask,
                        const dnatok_encode_opts &o) {
    int rc = check_inputs(v, d_bytes, nbytes, d_offsets, n, d_out_offsets, o);
    if (rc) return rc;
    if (ids_capacity < 0) return set_error(DNATOK_EINVAL, "negative size");
    if (ids_capacity > 0 && !d_ids) return set_error(DNATOK_EINVAL, "null ids");
    if ((reinterpret_cast<uintptr_t>(d_ids) & 3) != 0) return set_error(DNATOK_EINVAL, "ids must be 4-byte aligned");
    if (o.layout == DNATOK_PADDED && !d_mask) return set_error(DNATOK_EINVAL, "PADDED needs a mask buffer");
    return check_padded_cap(n, ids_capacity, o, "ids_capacity");
}

int dnatok_encode(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets, int32_t n,
                  int32_t *d_ids, int64_t ids_capacity, int64_t *d_out_offsets, int8_t *d_mask,
                  const dnatok_encode_opts *opts, void *stream) {
    dnatok_encode_opts o = {};
    if (opts) o = *opts;
    int rc = check_encode(v, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets, d_mask, o);
    if (rc) return rc;
    clear_error();
    if (v->kind == DNATOK_BPE)
        return launch_bpe_encode(v, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets, d_mask, o,
                                 static_cast<hipStream_t>(stream));
    if (o.variant)
        return launch_encode_variant(v, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets, d_mask, o,
                                     static_cast<hipStream_t>(stream));
    return launch_encode(v, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets, d_mask, o,
                         static_cast<hipStream_t>(stream));
}

int dnatok_encode_noalloc(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                          int32_t n, int32_t *d_ids, int64_t ids_capacity, int64_t *d_out_offsets, int8_t *d_mask,
                          const dnatok_encode_opts *opts, void *stream) {
    dnatok_encode_opts o = {};
    if (opts) o = *opts;
    int rc = check_encode(v, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets, d_mask, o);
    if (rc) return rc;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace *ws = nullptr;
    rc = fixed_workspace(s, &ws);
    if (rc) return rc;
    clear_error();
    FixedWorkspaceScope scope(ws);
    if (v->kind == DNATOK_BPE)
        return launch_bpe_encode(v, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets, d_mask, o, s);
    if (o.variant)
        return launch_encode_variant(v, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets, d_mask, o,
                                     s);
    return launch_encode(v, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets, d_mask, o, s);
}

int dnatok_encode_multi(const dnatok_vocab *const *vocabs, int32_t n_vocabs, const uint8_t *d_bytes, int64_t nbytes,
                        const int64_t *d_offsets, int32_t n, int32_t *const *d_ids, const int64_t *ids_capacity,
                        int64_t *const *d_out_offsets, int8_t *const *d_mask, const dnatok_encode_opts *opts,
                        void *stream) {
    if (!vocabs || !d_ids || !ids_capacity || !d_out_offsets || !d_mask || !opts)
        return set_error(DNATOK_EINVAL, "null argument array");
    if (n_vocabs < 1 || n_vocabs > 8) return set_error(DNATOK_EINVAL, "n_vocabs must be 1..8");
    for (int32_t i = 0; i < n_vocabs; ++i) {
        int rc = check_encode(vocabs[i], d_bytes, nbytes, d_offsets, n, d_ids[i], ids_capacity[i], d_out_offsets[i],
                              d_mask[i], opts[i]);
        if (rc) return rc;
        if (n_vocabs > 1 && vocabs[i]->kind != DNATOK_KMER)
            return set_error(DNATOK_EVOCAB, "several vocabularies in one pass must all be k-mer vocabularies");
        if (n_vocabs > 1 && opts[i].variant)
            return set_error(DNATOK_EINVAL, "encode variants take one vocabulary per call");
        if (opts[i].add_cls_sep != opts[0].add_cls_sep || opts[i].layout != opts[0].layout ||
            opts[i].pad_side != opts[0].pad_side)
            return set_error(DNATOK_EINVAL, "options differ in more than pad_to and offset_base");
    }
    clear_error();
    if (n_vocabs == 1) return dnatok_encode(vocabs[0], d_bytes, nbytes, d_offsets, n, d_ids[0], ids_capacity[0],
                                            d_out_offsets[0], d_mask[0], &opts[0], stream);
    return launch_encode_multi(vocabs, n_vocabs, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets,
                               d_mask, opts, static_cast<hipStream_t>(stream));
}

static int check_table(const void *d_table, int64_t n_rows, int64_t row_bytes, const void *d_out, int64_t out_rows) {
    if (row_bytes < 1 || row_bytes > (1 << 20)) return set_error(DNATOK_EINVAL, "row_bytes must be 1 .. 2^20");
    if (n_rows < 1 || !d_table) return set_error(DNATOK_EINVAL, "an embedding table is required");
    if (out_rows < 0) return set_error(DNATOK_EINVAL, "negative size");
    if (out_rows > 0 && !d_out) return set_error(DNATOK_EINVAL, "null output");
    return DNATOK_OK;
}

int dnatok_embed(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets, int32_t n,
                 const void *d_table, int64_t n_rows, int64_t row_bytes, void *d_out, int64_t out_rows,
                 int64_t *d_out_offsets, int32_t *d_ids, int8_t *d_mask, const dnatok_encode_opts *opts,
                 void *stream) {
    dnatok_encode_opts o = {};
    if (opts) o = *opts;
    if (!v) return set_error(DNATOK_EINVAL, "null vocabulary");
    if (v->kind == DNATOK_BPE) return set_error(DNATOK_EVOCAB, "BPE: encode, then dnatok_embed_ids");
    int rc = check_table(d_table, n_rows, row_bytes, d_out, out_rows);
    if (rc) return rc;
    if (n_rows < v->vocab_size)
        return set_error(DNATOK_EINVAL, "table has %lld rows, the vocabulary %d ids", (long long)n_rows, v->vocab_size);
    rc = check_inputs(v, d_bytes, nbytes, d_offsets, n, d_out_offsets, o);
    if (rc) return rc;
    if ((reinterpret_cast<uintptr_t>(d_ids) & 3) != 0) return set_error(DNATOK_EINVAL, "ids must be 4-byte aligned");
    rc = check_padded_cap(n, out_rows, o, "out_rows");
    if (rc) return rc;
    clear_error();
    return launch_embed(v, d_bytes, nbytes, d_offsets, n, d_table, n_rows, row_bytes, d_out, out_rows, d_out_offsets,
                        d_ids, d_mask, o, static_cast<hipStream_t>(stream));
}

int dnatok_embed_ids(const int32_t *d_ids, int64_t n_ids, const void *d_table, int64_t n_rows, int64_t row_bytes,
                     void *d_out, void *stream) {
    if (n_ids < 0) return set_error(DNATOK_EINVAL, "negative size");
    if (n_ids > 0 && !d_ids) return set_error(DNATOK_EINVAL, "null ids");
    if ((reinterpret_cast<uintptr_t>(d_ids) & 3) != 0) return set_error(DNATOK_EINVAL, "ids must be 4-byte aligned");
    int rc = check_table(d_table, n_rows, row_bytes, d_out, n_ids);
    if (rc) return rc;
    clear_error();
    if (n_ids == 0) return DNATOK_OK;
    return launch_embed_ids(d_ids, nullptr, n_ids, d_table, n_rows, row_bytes, d_out,
                            static_cast<hipStream_t>(stream));
}

int dnatok_sync_status(void *stream, uint32_t *flags) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    DNATOK_HIP(hipStreamSynchronize(s));
    uint32_t f = 0;
    Workspace *ws = find_workspace(s);
    if (ws && ws->d_hdr) {
        DNATOK_HIP(hipMemcpy(&f, ws->d_hdr + HDR_ERR, sizeof(f), hipMemcpyDeviceToHost));
        DNATOK_HIP(hipMemsetAsync(ws->d_hdr + HDR_ERR, 0, sizeof(uint32_t), s));
        DNATOK_HIP(hipStreamSynchronize(s));
    }
    uint32_t ff = 0;
    int rc = take_fixed_flags(s, &ff);
    if (rc) return rc;
    if (flags) *flags = f | ff;
    return DNATOK_OK;
}

int dnatok_decode(const dnatok_vocab *v, const int32_t *d_ids, int64_t n_ids, const int64_t *d_offsets, int32_t n,
                  uint8_t *d_out, int64_t out_capacity, int64_t *d_out_offsets, void *stream) {
    if (!v) return set_error(DNATOK_EINVAL, "null vocabulary");
    if (v->kind == DNATOK_LUT256) return set_error(DNATOK_EVOCAB, "decode is not defined for LUT256");
    if (n < 0 || n_ids < 0 || out_capacity < 0) return set_error(DNATOK_EINVAL, "negative size");
    if (!d_offsets || !d_out_offsets) return set_error(DNATOK_EINVAL, "offsets and out_offsets are required");
    if (n_ids > 0 && !d_ids) return set_error(DNATOK_EINVAL, "null ids");
    if (out_capacity > 0 && !d_out) return set_error(DNATOK_EINVAL, "null output");
    int dev = 0;
    DNATOK_HIP(hipGetDevice(&dev));
    if (dev != v->device) return set_error(DNATOK_EINVAL, "vocabulary lives on device %d, current is %d", v->device, dev);
    clear_error();
    return launch_decode(v, d_ids, n_ids, d_offsets, n, d_out, out_capacity, d_out_offsets,
                         static_cast<hipStream_t>(stream));
}

}  // extern "C"
