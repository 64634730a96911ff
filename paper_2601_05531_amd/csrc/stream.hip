// Pinned host-to-device stream overlapped with encode (dnatok_stream_*).
//
// Paper: Design, "Pipelined streaming" (separate streams, pre-allocated
// device buffers, events ordering transfers against compute) applied to the
// bytes path: raw bytes cross the host link once and are encoded on the
// device. Window cutting is host-side arithmetic over record ends; every
// device step is enqueued asynchronously.
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "hostbook.hpp"

namespace {

constexpr int64_t kAlign = 256;

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

}  // namespace

struct dnatok_stream {
    const dnatok_vocab *v = nullptr;
    dnatok_stream_opts o{};
    hipStream_t compute = nullptr;
    hipStream_t copy = nullptr;  // == compute when overlap == 0
    bool own_copy = false;
    int64_t pre = 0;  // prefix area per slot (>= window - 1, aligned)
    std::vector<uint8_t *> d_slot;
    std::vector<int64_t *> d_offs;
    std::vector<int64_t *> h_offs;  // pinned staging of window offsets, per slot
    std::vector<int64_t> offs_cap;  // entries
    std::vector<hipEvent_t> ev_copied, ev_free;
    std::vector<bool> copied_pending;
    int64_t *d_tail_offs = nullptr;  // flush: offsets of the final window
    int64_t *h_tail_offs = nullptr;
    int32_t *d_ids = nullptr;
    int64_t *d_woff = nullptr;
    // progress
    int64_t chunk = 0;
    int64_t n_windows = 0, n_tokens = 0, n_bytes = 0;
    int prev_slot = -1;
    const uint8_t *carry_src = nullptr;  // device bytes of the unfinished window
    int64_t carry_len = 0;
    bool failed = false, flushed = false;
};

namespace dnatok {

// Tokens of one window of L bases.
static int64_t window_tokens(const dnatok_vocab *v, int64_t L, int32_t cls) {
    const int64_t k = (v->kind == DNATOK_KMER) ? v->k : 1;
    return (L + k - 1) / k + 2 * cls;
}

static void free_stream(dnatok_stream *s) {
    for (auto p : s->d_slot) if (p) (void)hipFree(p);
    for (auto p : s->d_offs) if (p) (void)hipFree(p);
    for (auto p : s->h_offs) if (p) (void)hipHostFree(p);
    for (auto e : s->ev_copied) if (e) (void)hipEventDestroy(e);
    for (auto e : s->ev_free) if (e) (void)hipEventDestroy(e);
    if (s->d_tail_offs) (void)hipFree(s->d_tail_offs);
    if (s->h_tail_offs) (void)hipHostFree(s->h_tail_offs);
    if (s->d_ids) (void)hipFree(s->d_ids);
    if (s->d_woff) (void)hipFree(s->d_woff);
    if (s->own_copy && s->copy) (void)hipStreamDestroy(s->copy);
    delete s;
}

// Grow slot `i`'s offset staging to hold `entries` int64 (outside any
// in-flight use: the slot's previous copy is complete when this is called).
static int ensure_offs(dnatok_stream *s, int i, int64_t entries) {
    if (entries <= s->offs_cap[i]) return DNATOK_OK;
    int64_t cap = std::max<int64_t>(entries, 2 * s->offs_cap[i]);
    if (s->d_offs[i]) DNATOK_HIP(hipFree(s->d_offs[i]));
    if (s->h_offs[i]) DNATOK_HIP(hipHostFree(s->h_offs[i]));
    s->d_offs[i] = nullptr;
    s->h_offs[i] = nullptr;
    s->offs_cap[i] = 0;
    void *p = nullptr;
    DNATOK_HIP(dev_alloc(&p, sizeof(int64_t) * (size_t)cap));
    s->d_offs[i] = static_cast<int64_t *>(p);
    DNATOK_HIP(host_alloc(&p, sizeof(int64_t) * (size_t)cap));
    s->h_offs[i] = static_cast<int64_t *>(p);
    s->offs_cap[i] = cap;
    return DNATOK_OK;
}

}  // namespace dnatok

using namespace dnatok;

extern "C" {

int dnatok_stream_create(const dnatok_vocab *v, const dnatok_stream_opts *opts, void *compute_stream,
                         dnatok_stream **out) {
    if (!v || !opts || !out) return set_error(DNATOK_EINVAL, "null argument");
    *out = nullptr;
    if (v->kind == DNATOK_BPE)
        return set_error(DNATOK_EVOCAB, "streams need token counts known on the host (SINGLE, LUT256, KMER)");
    const dnatok_stream_opts &o = *opts;
    if (o.window < 1 || o.chunk_bytes < 1 || o.n_slots < 2 || o.n_slots > 16 || o.max_tokens < 0 ||
        o.max_windows < 0)
        return set_error(DNATOK_EINVAL, "bad stream options");
    int dev = 0;
    DNATOK_HIP(hipGetDevice(&dev));
    if (dev != v->device) return set_error(DNATOK_EINVAL, "vocabulary lives on device %d, current is %d", v->device, dev);
    dnatok_stream *s = new dnatok_stream();
    s->v = v;
    s->o = o;
    s->compute = static_cast<hipStream_t>(compute_stream);
    s->pre = round_up(o.window, kAlign);
    int rc = DNATOK_OK;
    auto fail = [&](int code) {
        free_stream(s);
        return code;
    };
    if (o.overlap) {
        hipError_t e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(set_error(DNATOK_EDEVICE, "copy stream: %s", hipGetErrorString(e)));
        s->own_copy = true;
    } else {
        s->copy = s->compute;
    }
    const int n = o.n_slots;
    s->d_slot.assign(n, nullptr);
    s->d_offs.assign(n, nullptr);
    s->h_offs.assign(n, nullptr);
    s->offs_cap.assign(n, 0);
    s->ev_copied.assign(n, nullptr);
    s->ev_free.assign(n, nullptr);
    s->copied_pending.assign(n, false);
    const int64_t per_chunk_windows = o.chunk_bytes / o.window + 64;
    for (int i = 0; i < n; ++i) {
        void *p = nullptr;
        hipError_t e = dev_alloc(&p, (size_t)(s->pre + round_up(o.chunk_bytes, kAlign) + kAlign));
        if (e != hipSuccess) return fail(set_error(DNATOK_ENOMEM, "slot %d: %s", i, hipGetErrorString(e)));
        s->d_slot[i] = static_cast<uint8_t *>(p);
        if ((rc = ensure_offs(s, i, per_chunk_windows + 1))) return fail(rc);
        if (hipEventCreateWithFlags(&s->ev_copied[i], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&s->ev_free[i], hipEventDisableTiming) != hipSuccess)
            return fail(set_error(DNATOK_EDEVICE, "event creation failed"));
    }
    void *p = nullptr;
    if (dev_alloc(&p, 2 * sizeof(int64_t)) != hipSuccess) return fail(set_error(DNATOK_ENOMEM, "tail offsets"));
    s->d_tail_offs = static_cast<int64_t *>(p);
    if (host_alloc(&p, 2 * sizeof(int64_t)) != hipSuccess)
        return fail(set_error(DNATOK_ENOMEM, "tail offsets"));
    s->h_tail_offs = static_cast<int64_t *>(p);
    if (dev_alloc(&p, sizeof(int32_t) * (size_t)std::max<int64_t>(o.max_tokens, 1)) != hipSuccess)
        return fail(set_error(DNATOK_ENOMEM, "output ids (%lld tokens)", (long long)o.max_tokens));
    s->d_ids = static_cast<int32_t *>(p);
    if (dev_alloc(&p, sizeof(int64_t) * (size_t)(o.max_windows + 1)) != hipSuccess)
        return fail(set_error(DNATOK_ENOMEM, "window offsets"));
    s->d_woff = static_cast<int64_t *>(p);
    *out = s;
    return dnatok_stream_reset(s);
}

int dnatok_stream_reset(dnatok_stream *s) {
    if (!s) return set_error(DNATOK_EINVAL, "null stream");
    DNATOK_HIP(hipStreamSynchronize(s->compute));
    if (s->own_copy) DNATOK_HIP(hipStreamSynchronize(s->copy));
    s->chunk = 0;
    s->n_windows = s->n_tokens = s->n_bytes = 0;
    s->prev_slot = -1;
    s->carry_src = nullptr;
    s->carry_len = 0;
    s->failed = s->flushed = false;
    std::fill(s->copied_pending.begin(), s->copied_pending.end(), false);
    // out_offsets[0] = 0 even when no window is ever written
    DNATOK_HIP(hipMemsetAsync(s->d_woff, 0, sizeof(int64_t), s->compute));
    DNATOK_HIP(hipStreamSynchronize(s->compute));
    return DNATOK_OK;
}

int dnatok_stream_push(dnatok_stream *s, const uint8_t *h, int64_t nbytes, const int64_t *ends, int32_t n_ends) {
    if (!s) return set_error(DNATOK_EINVAL, "null stream");
    if (s->failed || s->flushed) return set_error(DNATOK_ESTATE, "stream is %s", s->failed ? "failed" : "flushed");
    // Any failure below leaves the windows pushed so far intact and poisons
    // the stream: a skipped chunk would silently shift every later window.
    auto reject = [&](int code) {
        s->failed = true;
        return code;
    };
    const dnatok_stream_opts &o = s->o;
    if (nbytes < 0 || nbytes > o.chunk_bytes || (nbytes > 0 && !h) || n_ends < 0 || (n_ends > 0 && !ends))
        return reject(set_error(DNATOK_EINVAL, "bad push arguments"));
    for (int32_t i = 0; i < n_ends; ++i)
        if (ends[i] < 0 || ends[i] > nbytes || (i > 0 && ends[i] < ends[i - 1]))
            return reject(set_error(DNATOK_EINVAL, "record_ends must be non-decreasing within [0, nbytes]"));
    if (nbytes > 0) {
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, h) != hipSuccess || attr.type != hipMemoryTypeHost) {
            (void)hipGetLastError();
            return reject(set_error(DNATOK_EINVAL, "pushed bytes must be pinned host memory"));
        }
    }
    const int slot = (int)(s->chunk % o.n_slots);
    // The offsets staging of this slot was last read by a copy n_slots chunks ago.
    if (s->copied_pending[slot]) DNATOK_HIP(hipEventSynchronize(s->ev_copied[slot]));

    // Cut windows over S = carry ++ chunk (coordinates from the carry's first byte).
    const int64_t cl = s->carry_len, slen = cl + nbytes;
    std::vector<int64_t> cuts;
    const int64_t cur = cut_windows(cl, nbytes, o.window, ends, n_ends, cuts);
    const int64_t nwin = (int64_t)cuts.size() - 1;
    int64_t toks = 0;
    for (int64_t w = 0; w < nwin; ++w) toks += window_tokens(s->v, cuts[w + 1] - cuts[w], o.add_cls_sep);
    if (s->n_windows + nwin > o.max_windows)
        return reject(set_error(DNATOK_ETOOSMALL, "max_windows (%lld) exceeded", (long long)o.max_windows));
    if (s->n_tokens + toks > o.max_tokens)
        return reject(set_error(DNATOK_ETOOSMALL, "max_tokens (%lld) exceeded", (long long)o.max_tokens));
    if (nwin + 1 > s->offs_cap[slot]) {
        // growing frees the slot's offsets, which an earlier encode may still read
        DNATOK_HIP(hipStreamSynchronize(s->compute));
        if (s->own_copy) DNATOK_HIP(hipStreamSynchronize(s->copy));
    }
    int rc = ensure_offs(s, slot, nwin + 1);
    if (rc) return reject(rc);
    std::copy(cuts.begin(), cuts.end(), s->h_offs[slot]);

    uint8_t *data = s->d_slot[slot] + s->pre;  // the chunk lands here
    auto fail = reject;
    // Copy stream: wait until the slot is free, then bytes and offsets.
    if (hipStreamWaitEvent(s->copy, s->ev_free[slot], 0) != hipSuccess ||
        (nbytes > 0 && hipMemcpyAsync(data, h, (size_t)nbytes, hipMemcpyHostToDevice, s->copy) != hipSuccess) ||
        hipMemcpyAsync(s->d_offs[slot], s->h_offs[slot], sizeof(int64_t) * (size_t)(nwin + 1), hipMemcpyHostToDevice,
                       s->copy) != hipSuccess ||
        hipEventRecord(s->ev_copied[slot], s->copy) != hipSuccess)
        return fail(set_error(DNATOK_EDEVICE, "enqueueing the chunk copy failed"));
    s->copied_pending[slot] = true;
    // Compute stream: wait for the copy, bring the unfinished window in front
    // of the chunk, release the previous slot, encode the complete windows.
    if (hipStreamWaitEvent(s->compute, s->ev_copied[slot], 0) != hipSuccess)
        return fail(set_error(DNATOK_EDEVICE, "stream wait failed"));
    if (cl > 0 && hipMemcpyAsync(data - cl, s->carry_src, (size_t)cl, hipMemcpyDeviceToDevice, s->compute) != hipSuccess)
        return fail(set_error(DNATOK_EDEVICE, "carry copy failed"));
    if (s->prev_slot >= 0 && hipEventRecord(s->ev_free[s->prev_slot], s->compute) != hipSuccess)
        return fail(set_error(DNATOK_EDEVICE, "event record failed"));
    if (nwin > 0) {
        dnatok_encode_opts eo = {};
        eo.add_cls_sep = o.add_cls_sep;
        eo.layout = DNATOK_PACKED;
        eo.offset_base = s->n_tokens;
        rc = launch_encode(s->v, data - cl, slen, s->d_offs[slot], (int32_t)nwin, s->d_ids + s->n_tokens, toks,
                           s->d_woff + s->n_windows, nullptr, eo, s->compute);
        if (rc) return fail(rc);
    }
    s->n_windows += nwin;
    s->n_tokens += toks;
    s->n_bytes += nbytes;
    s->carry_src = data - cl + cur;
    s->carry_len = slen - cur;
    s->prev_slot = slot;
    s->chunk += 1;
    return DNATOK_OK;
}

int dnatok_stream_flush(dnatok_stream *s, dnatok_stream_result *out) {
    if (!s) return set_error(DNATOK_EINVAL, "null stream");
    if (s->failed || s->flushed) return set_error(DNATOK_ESTATE, "stream is %s", s->failed ? "failed" : "flushed");
    const dnatok_stream_opts &o = s->o;
    if (s->carry_len > 0) {
        const int64_t toks = window_tokens(s->v, s->carry_len, o.add_cls_sep);
        if (s->n_windows + 1 > o.max_windows || s->n_tokens + toks > o.max_tokens) {
            s->failed = true;
            return set_error(DNATOK_ETOOSMALL, "the final window does not fit the output buffers");
        }
        s->h_tail_offs[0] = 0;
        s->h_tail_offs[1] = s->carry_len;
        DNATOK_HIP(hipMemcpyAsync(s->d_tail_offs, s->h_tail_offs, 2 * sizeof(int64_t), hipMemcpyHostToDevice,
                                  s->compute));
        dnatok_encode_opts eo = {};
        eo.add_cls_sep = o.add_cls_sep;
        eo.layout = DNATOK_PACKED;
        eo.offset_base = s->n_tokens;
        int rc = launch_encode(s->v, s->carry_src, s->carry_len, s->d_tail_offs, 1, s->d_ids + s->n_tokens, toks,
                               s->d_woff + s->n_windows, nullptr, eo, s->compute);
        if (rc) {
            s->failed = true;
            return rc;
        }
        s->n_windows += 1;
        s->n_tokens += toks;
        s->carry_len = 0;
    }
    DNATOK_HIP(hipStreamSynchronize(s->compute));
    if (s->own_copy) DNATOK_HIP(hipStreamSynchronize(s->copy));
    s->flushed = true;
    if (out) {
        out->d_ids = s->d_ids;
        out->d_window_offsets = s->d_woff;
        out->n_windows = s->n_windows;
        out->n_tokens = s->n_tokens;
        out->n_bytes = s->n_bytes;
    }
    return DNATOK_OK;
}

int dnatok_stream_destroy(dnatok_stream *s) {
    if (!s) return set_error(DNATOK_EINVAL, "null stream");
    (void)hipStreamSynchronize(s->compute);
    if (s->own_copy) (void)hipStreamSynchronize(s->copy);
    free_stream(s);
    return DNATOK_OK;
}

}  // extern "C"
