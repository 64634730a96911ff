// The IDs path: host mapping into pinned staging, staged id transfer,
// on-device widening and the embedder, sequential or pipelined.
//
// Paper: Design, "IDs path (CPU staging)" (a vectorized host map through the
// 256-entry table into persistent pinned buffers, non-blocking copies of 32-
// or 64-bit ids, on-device promotion of int32 to int64), the host-side
// branch of the EmbedFromStrings algorithm (left padding to token_len,
// micro-batches of b = min(B_emb, max(1, floor(M / T'))) rows, one embedder
// call per micro-batch) and "Pipelined streaming" (two streams, ping-pong
// device buffers, events ordering copies against compute).
//
// MI355X mapping: the host map runs on a persistent worker pool, rows split
// evenly; copies come from one pinned staging area sized for the whole
// batch, so the host never waits on a buffer; the widen kernel moves 16 bytes
// in and 32 bytes out per thread; the embedder is the library's table-row
// lookup reading the int64 ids.
#include <chrono>
#include <memory>
#include <thread>

#include "common.hpp"
#include "hostbook.hpp"

namespace dnatok {
namespace {

constexpr int NTW = 256;
constexpr int64_t kDefaultBudget = 1 << 20;  // the paper's default tokens per embedder call

// dst[i] = (int64) src[i], i < n. Four ids per thread (one 16-byte load, two
// 16-byte stores) when both pointers are 16-byte aligned.
__global__ __launch_bounds__(NTW) void k_widen(const int32_t *__restrict__ src, int64_t *__restrict__ dst, int64_t n,
                                                int32_t vec) {
    const int64_t stride = (int64_t)gridDim.x * NTW;
    const int64_t t0 = (int64_t)blockIdx.x * NTW + threadIdx.x;
    int64_t done = 0;
    if (vec) {
        typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
        typedef int64_t i64x2 __attribute__((ext_vector_type(2)));
        const int64_t n4 = n >> 2;
        const i32x4 *s4 = reinterpret_cast<const i32x4 *>(src);
        i64x2 *d2 = reinterpret_cast<i64x2 *>(dst);
        for (int64_t i = t0; i < n4; i += stride) {
            const i32x4 v = __builtin_nontemporal_load(s4 + i);
            const i64x2 a = {(int64_t)v[0], (int64_t)v[1]}, b = {(int64_t)v[2], (int64_t)v[3]};
            __builtin_nontemporal_store(a, d2 + 2 * i);
            __builtin_nontemporal_store(b, d2 + 2 * i + 1);
        }
        done = n4 << 2;
    }
    for (int64_t i = done + t0; i < n; i += stride) dst[i] = (int64_t)src[i];
}

int launch_widen(const int32_t *src, int64_t *dst, int64_t n, hipStream_t stream) {
    if (n <= 0) return DNATOK_OK;
    const int32_t vec = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0;
    const int64_t per = vec ? 4 : 1;
    int64_t g = (n / per + NTW - 1) / NTW;
    g = std::max<int64_t>(1, std::min<int64_t>(g, (int64_t)device_cu_count() * 8));
    hipLaunchKernelGGL(k_widen, dim3((unsigned)g), dim3(NTW), 0, stream, src, dst, n, vec);
    DNATOK_HIP(hipGetLastError());
    return DNATOK_OK;
}

int default_threads() {
    unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(h ? h : 1u, 16u));
}

// Rows [0, n) cut into `parts` near-equal ranges: part p is [lo, hi).
void part_rows(int64_t n, int parts, int p, int64_t *lo, int64_t *hi) {
    *lo = n * p / parts;
    *hi = n * (p + 1) / parts;
}

void map_parallel(WorkerPool &pool, const int32_t *lut, int32_t pad_id, const uint8_t *src, int64_t n_rows,
                  int64_t row_len, int64_t token_len, int32_t width, void *dst) {
    const int parts = (int)std::max<int64_t>(1, std::min<int64_t>(n_rows, pool.size()));
    pool.run(parts, [&](int p) {
        int64_t lo, hi;
        part_rows(n_rows, parts, p, &lo, &hi);
        if (width == 4)
            map_rows_to_ids(lut, pad_id, src, lo, hi, row_len, token_len, static_cast<int32_t *>(dst));
        else
            map_rows_to_ids(lut, pad_id, src, lo, hi, row_len, token_len, static_cast<int64_t *>(dst));
    });
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace
}  // namespace dnatok

using namespace dnatok;

struct dnatok_ids {
    int device = 0;
    dnatok_ids_opts o{};
    int32_t lut[256];
    int32_t pad_id = 0;
    hipStream_t compute = nullptr;
    hipStream_t copy = nullptr;  // pipelined form only
    hipEvent_t copied[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> timing;  // two per micro-batch: around its copy
    void *h_stage = nullptr;
    int64_t h_stage_bytes = 0;
    void *d_stage[2] = {nullptr, nullptr};  // copy targets (width bytes per id)
    int64_t d_stage_bytes = 0;
    int64_t *d_wide[2] = {nullptr, nullptr};  // int32 staging: widened ids
    int64_t d_wide_bytes = 0;
    std::unique_ptr<WorkerPool> pool;

    ~dnatok_ids() {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(device);
        if (compute) (void)hipStreamSynchronize(compute);
        if (copy) {
            (void)hipStreamSynchronize(copy);
            (void)hipStreamDestroy(copy);
        }
        for (int i = 0; i < 2; ++i) {
            if (copied[i]) (void)hipEventDestroy(copied[i]);
            if (freed[i]) (void)hipEventDestroy(freed[i]);
            if (d_stage[i]) (void)hipFree(d_stage[i]);
            if (d_wide[i]) (void)hipFree(d_wide[i]);
        }
        for (hipEvent_t e : timing) (void)hipEventDestroy(e);
        if (h_stage) (void)hipHostFree(h_stage);
        (void)hipSetDevice(prev);
    }
};

namespace {

// Grow the staging and device buffers to hold a run of n_rows rows of T' ids
// in micro-batches of b rows (synchronous: outside any timed region).
int ensure_buffers(dnatok_ids *p, int64_t n_rows, int64_t T, int64_t b, int64_t n_micro) {
    const int64_t w = p->o.width;
    const int64_t hb = n_rows * T * w;
    if (hb > p->h_stage_bytes) {
        DNATOK_HIP(hipStreamSynchronize(p->compute));
        if (p->copy) DNATOK_HIP(hipStreamSynchronize(p->copy));
        if (p->h_stage) DNATOK_HIP(hipHostFree(p->h_stage));
        p->h_stage = nullptr;
        p->h_stage_bytes = 0;
        DNATOK_HIP(host_alloc(&p->h_stage, (size_t)std::max<int64_t>(hb, 256)));
        p->h_stage_bytes = std::max<int64_t>(hb, 256);
    }
    const int64_t nbuf = p->o.overlap ? 2 : 1;
    const int64_t db = b * T * w;
    if (db > p->d_stage_bytes) {
        DNATOK_HIP(hipStreamSynchronize(p->compute));
        if (p->copy) DNATOK_HIP(hipStreamSynchronize(p->copy));
        for (int i = 0; i < 2; ++i) {
            if (p->d_stage[i]) DNATOK_HIP(hipFree(p->d_stage[i]));
            p->d_stage[i] = nullptr;
        }
        p->d_stage_bytes = 0;
        for (int64_t i = 0; i < nbuf; ++i) DNATOK_HIP(dev_alloc(&p->d_stage[i], (size_t)db));
        p->d_stage_bytes = db;
    }
    const int64_t wb = (w == 4) ? b * T * 8 : 0;
    if (wb > p->d_wide_bytes) {
        DNATOK_HIP(hipStreamSynchronize(p->compute));
        for (int i = 0; i < 2; ++i) {
            if (p->d_wide[i]) DNATOK_HIP(hipFree(p->d_wide[i]));
            p->d_wide[i] = nullptr;
        }
        p->d_wide_bytes = 0;
        for (int64_t i = 0; i < nbuf; ++i) {
            void *q = nullptr;
            DNATOK_HIP(dev_alloc(&q, (size_t)wb));
            p->d_wide[i] = static_cast<int64_t *>(q);
        }
        p->d_wide_bytes = wb;
    }
    while ((int64_t)p->timing.size() < 2 * n_micro) {
        hipEvent_t e = nullptr;
        DNATOK_HIP(hipEventCreate(&e));
        p->timing.push_back(e);
    }
    return DNATOK_OK;
}

}  // namespace

extern "C" {

int dnatok_ids_map(const int32_t *lut256, int32_t pad_id, const uint8_t *h_bytes, int64_t n_rows, int64_t row_len,
                   int64_t token_len, int32_t width, void *h_out, int32_t threads) {
    if (!lut256) return set_error(DNATOK_EINVAL, "null table");
    if (n_rows < 0 || row_len < 0 || threads < 0) return set_error(DNATOK_EINVAL, "negative size");
    if (width != 4 && width != 8) return set_error(DNATOK_EINVAL, "width must be 4 or 8");
    if (token_len == 0) token_len = row_len;
    if (token_len < row_len) return set_error(DNATOK_EINVAL, "token_len %lld < row length %lld",
                                              (long long)token_len, (long long)row_len);
    if (n_rows > 0 && token_len > 0 && !h_out) return set_error(DNATOK_EINVAL, "null output");
    if (n_rows > 0 && row_len > 0 && !h_bytes) return set_error(DNATOK_EINVAL, "null input");
    clear_error();
    if (n_rows == 0 || token_len == 0) return DNATOK_OK;
    WorkerPool pool(threads > 0 ? std::min(threads, 64) : default_threads());
    map_parallel(pool, lut256, pad_id, h_bytes, n_rows, row_len, token_len, width, h_out);
    return DNATOK_OK;
}

int dnatok_ids_create(const dnatok_vocab *v, const dnatok_ids_opts *opts, void *compute_stream, dnatok_ids **out) {
    if (!v || !opts || !out) return set_error(DNATOK_EINVAL, "null argument");
    *out = nullptr;
    if (v->kind != DNATOK_SINGLE && v->kind != DNATOK_LUT256)
        return set_error(DNATOK_EVOCAB, "the IDs path maps bytes through a table: SINGLE or LUT256");
    if (opts->width != 4 && opts->width != 8) return set_error(DNATOK_EINVAL, "width must be 4 or 8");
    if (opts->overlap != 0 && opts->overlap != 1) return set_error(DNATOK_EINVAL, "overlap must be 0 or 1");
    if (opts->threads < 0 || opts->token_budget < 0 || opts->max_rows < 0)
        return set_error(DNATOK_EINVAL, "negative option");
    int dev = 0;
    DNATOK_HIP(hipGetDevice(&dev));
    if (dev != v->device) return set_error(DNATOK_EINVAL, "vocabulary lives on device %d, current is %d", v->device, dev);
    std::unique_ptr<dnatok_ids> p(new dnatok_ids());
    p->device = dev;
    p->o = *opts;
    if (p->o.token_budget == 0) p->o.token_budget = kDefaultBudget;
    p->pad_id = v->pad_id;
    DNATOK_HIP(hipMemcpy(p->lut, v->d_lut, sizeof(p->lut), hipMemcpyDeviceToHost));
    p->compute = static_cast<hipStream_t>(compute_stream);
    if (p->o.overlap) DNATOK_HIP(hipStreamCreateWithFlags(&p->copy, hipStreamNonBlocking));
    for (int i = 0; i < 2; ++i) {
        DNATOK_HIP(hipEventCreateWithFlags(&p->copied[i], hipEventDisableTiming));
        DNATOK_HIP(hipEventCreateWithFlags(&p->freed[i], hipEventDisableTiming));
    }
    Workspace *ws = nullptr;  // the embedder's error flags live in the compute stream's workspace
    int rc = get_workspace(p->compute, 1, &ws);
    if (rc) return rc;
    p->pool.reset(new WorkerPool(p->o.threads > 0 ? std::min(p->o.threads, 64) : default_threads()));
    clear_error();
    *out = p.release();
    return DNATOK_OK;
}

int dnatok_ids_run(dnatok_ids *p, const uint8_t *h_bytes, int64_t n_rows, int64_t row_len, int64_t token_len,
                   int64_t *d_ids, const void *d_table, int64_t n_table_rows, int64_t row_bytes, void *d_out,
                   dnatok_ids_result *res) {
    if (!p) return set_error(DNATOK_EINVAL, "null handle");
    if (n_rows < 0 || row_len < 0) return set_error(DNATOK_EINVAL, "negative size");
    if (token_len == 0) token_len = row_len;
    if (token_len < row_len) return set_error(DNATOK_EINVAL, "token_len %lld < row length %lld",
                                              (long long)token_len, (long long)row_len);
    if (!d_ids && !d_out) return set_error(DNATOK_EINVAL, "give d_ids, d_out or both");
    if (d_out && (!d_table || n_table_rows < 1 || row_bytes < 1 || row_bytes > (1 << 20)))
        return set_error(DNATOK_EINVAL, "d_out needs a table of n_table_rows >= 1 rows of 1 .. 2^20 bytes");
    if (n_rows > 0 && row_len > 0 && !h_bytes) return set_error(DNATOK_EINVAL, "null input");
    if ((reinterpret_cast<uintptr_t>(d_ids) & 7) != 0) return set_error(DNATOK_EINVAL, "d_ids must be 8-byte aligned");
    int dev = 0;
    DNATOK_HIP(hipGetDevice(&dev));
    if (dev != p->device) return set_error(DNATOK_EINVAL, "IDs path lives on device %d, current is %d", p->device, dev);
    const int64_t T = token_len;
    int64_t b = std::max<int64_t>(1, p->o.token_budget / std::max<int64_t>(T, 1));
    if (p->o.max_rows > 0) b = std::min(b, p->o.max_rows);
    b = std::max<int64_t>(1, std::min(b, n_rows));
    const int64_t n_micro = n_rows > 0 ? (n_rows + b - 1) / b : 0;
    dnatok_ids_result r{};
    r.rows = n_rows;
    r.token_len = T;
    r.micro_rows = b;
    r.n_micro = n_micro;
    clear_error();
    if (n_rows == 0 || T == 0) {
        if (res) *res = r;
        return DNATOK_OK;
    }
    int rc = ensure_buffers(p, n_rows, T, b, n_micro);
    if (rc) return rc;
    const int64_t w = p->o.width;

    const double t0 = now_s();
    // host map into the pinned staging, left-padded to T': every row first
    // (sequential form), or each micro-batch just before its copy, so that
    // the host maps micro-batch n + 1 while the copy engine moves n
    // (pipelined form; the copies and kernels are asynchronous)
    if (!p->o.overlap) {
        map_parallel(*p->pool, p->lut, p->pad_id, h_bytes, n_rows, row_len, T, (int32_t)w, p->h_stage);
        r.map_s = now_s() - t0;
    }

    const uint8_t *hs = static_cast<const uint8_t *>(p->h_stage);
    for (int64_t m = 0; m < n_micro; ++m) {
        const int64_t lo = m * b, rows = std::min(b, n_rows - lo), cells = rows * T;
        if (p->o.overlap) {
            const double tm = now_s();
            map_parallel(*p->pool, p->lut, p->pad_id, h_bytes + lo * row_len, rows, row_len, T, (int32_t)w,
                         static_cast<uint8_t *>(p->h_stage) + lo * T * w);
            r.map_s += now_s() - tm;
        }
        const int buf = p->o.overlap ? (int)(m & 1) : 0;
        // the ids the embedder reads: the caller's slice, else a ping-pong buffer
        int64_t *ids64 = d_ids ? d_ids + lo * T : (w == 8 ? static_cast<int64_t *>(p->d_stage[buf]) : p->d_wide[buf]);
        void *dst = (w == 8) ? static_cast<void *>(ids64) : p->d_stage[buf];
        const hipStream_t cs = p->o.overlap ? p->copy : p->compute;
        if (p->o.overlap && m >= 2) DNATOK_HIP(hipStreamWaitEvent(cs, p->freed[buf], 0));
        DNATOK_HIP(hipEventRecord(p->timing[2 * m], cs));
        DNATOK_HIP(hipMemcpyAsync(dst, hs + lo * T * w, (size_t)(cells * w), hipMemcpyHostToDevice, cs));
        DNATOK_HIP(hipEventRecord(p->timing[2 * m + 1], cs));
        r.h2d_bytes += cells * w;
        if (p->o.overlap) {
            DNATOK_HIP(hipEventRecord(p->copied[buf], cs));
            DNATOK_HIP(hipStreamWaitEvent(p->compute, p->copied[buf], 0));
        }
        if (w == 4) {
            rc = launch_widen(static_cast<const int32_t *>(p->d_stage[buf]), ids64, cells, p->compute);
            if (rc) return rc;
        }
        if (d_out) {
            rc = launch_embed_ids(nullptr, ids64, cells, d_table, n_table_rows, row_bytes,
                                  static_cast<uint8_t *>(d_out) + lo * T * row_bytes, p->compute);
            if (rc) return rc;
        }
        if (p->o.overlap) DNATOK_HIP(hipEventRecord(p->freed[buf], p->compute));
    }
    DNATOK_HIP(hipStreamSynchronize(p->compute));
    if (p->copy) DNATOK_HIP(hipStreamSynchronize(p->copy));
    r.total_s = now_s() - t0;
    double h2d = 0.0;
    for (int64_t m = 0; m < n_micro; ++m) {
        float ms = 0.0f;
        DNATOK_HIP(hipEventElapsedTime(&ms, p->timing[2 * m], p->timing[2 * m + 1]));
        h2d += ms * 1e-3;
    }
    r.h2d_s = h2d;
    if (res) *res = r;
    return DNATOK_OK;
}

int dnatok_ids_destroy(dnatok_ids *p) {
    if (!p) return set_error(DNATOK_EINVAL, "null handle");
    delete p;
    return DNATOK_OK;
}

}  // extern "C"
