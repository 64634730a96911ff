// Per-vocabulary tuning, the autotuner and captured encode graphs.
//
// The paper's batch and length sweeps (Results, "Encoding Throughput";
// Discussion, "Performance Characteristics and Scaling Behavior") show the
// encode's speed depending on how work is cut into launches and tiles; here
// the cut is chosen by timing candidates on the caller's own batch, and a
// fixed encode can be replayed from a HIP graph without per-launch host work.
#include <algorithm>
#include <vector>

#include "common.hpp"

using namespace dnatok;

namespace {

bool pow2_in(int32_t x, int32_t lo, int32_t hi) { return x >= lo && x <= hi && (x & (x - 1)) == 0; }

int check_tuning(const dnatok_tuning &t) {
    if (t.tile_bytes != 0 && !pow2_in(t.tile_bytes, 4096, 65536))
        return set_error(DNATOK_EINVAL, "tile_bytes must be 0 or a power of two in [4096, 65536]");
    if (t.blocks_per_cu < 0 || t.blocks_per_cu > 64) return set_error(DNATOK_EINVAL, "blocks_per_cu out of range");
    if (t.bpe_item_bytes != 0 && !pow2_in(t.bpe_item_bytes, kBpeItemBytesMin, 65536))
        return set_error(DNATOK_EINVAL, "bpe_item_bytes must be 0 or a power of two in [1024, 65536]");
    if (t.bpe_max_waves != 0 && t.bpe_max_waves != 1 && t.bpe_max_waves != 2 && t.bpe_max_waves != 4 &&
        t.bpe_max_waves != 8)
        return set_error(DNATOK_EINVAL, "bpe_max_waves must be 0, 1, 2, 4 or 8");
    if (t.spread < 0 || t.spread > 100) return set_error(DNATOK_EINVAL, "spread must be 0..100");
    if (t.bands < 0 || t.bands > 3) return set_error(DNATOK_EINVAL, "bands must be 0, 1, 2 or 3");
    return DNATOK_OK;
}

void store(dnatok_vocab *v, const dnatok_tuning &t) {
    v->tune_tile.store(t.tile_bytes, std::memory_order_relaxed);
    v->tune_blocks.store(t.blocks_per_cu, std::memory_order_relaxed);
    v->tune_item.store(t.bpe_item_bytes, std::memory_order_relaxed);
    v->tune_waves.store(t.bpe_max_waves, std::memory_order_relaxed);
    v->tune_spread.store(t.spread, std::memory_order_relaxed);
    v->tune_bands.store(t.bands, std::memory_order_relaxed);
}

dnatok_tuning load(const dnatok_vocab *v) {
    dnatok_tuning t;
    t.tile_bytes = v->tune_tile.load(std::memory_order_relaxed);
    t.blocks_per_cu = v->tune_blocks.load(std::memory_order_relaxed);
    t.bpe_item_bytes = v->tune_item.load(std::memory_order_relaxed);
    t.bpe_max_waves = v->tune_waves.load(std::memory_order_relaxed);
    t.spread = v->tune_spread.load(std::memory_order_relaxed);
    t.bands = v->tune_bands.load(std::memory_order_relaxed);
    return t;
}

}  // namespace

struct dnatok_graph {
    hipStream_t stream = nullptr;  // capture stream; owns the graph's workspace
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

int dnatok_get_tuning(const dnatok_vocab *v, dnatok_tuning *out) {
    if (!v || !out) return set_error(DNATOK_EINVAL, "null argument");
    *out = load(v);
    return DNATOK_OK;
}

int dnatok_set_tuning(dnatok_vocab *v, const dnatok_tuning *t) {
    if (!v || !t) return set_error(DNATOK_EINVAL, "null argument");
    int rc = check_tuning(*t);
    if (rc) return rc;
    store(v, *t);
    return DNATOK_OK;
}

}  // extern "C"

namespace {

// Times every candidate tiling of v with `run` (one encode on `st`): one
// warm-up sample and `reps` timed samples of 4 launches each, median; keeps the fastest in v.
template <class Run>
int autotune_loop(dnatok_vocab *v, hipStream_t st, int32_t reps, bool padded, Run run, dnatok_tuning *best,
                  float *best_ms) {
    if (!v) return set_error(DNATOK_EINVAL, "null vocabulary");
    if (reps < 1 || reps > 100) return set_error(DNATOK_EINVAL, "reps must be 1..100");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return set_error(DNATOK_ESTATE, "autotune cannot run during graph capture");
    std::vector<dnatok_tuning> cand;
    if (v->kind == DNATOK_BPE) {
        for (int32_t S : {2048, 4096, 8192, 16384, 32768})
            for (int32_t w : {8, 4, 2, 1}) cand.push_back(dnatok_tuning{0, 0, S, w, 0, 0});
    } else {
        for (int32_t tile : {4096, 8192, 16384, 32768, 65536})
            for (int32_t b : {0, 1, 2, 4}) cand.push_back(dnatok_tuning{tile, b, 0, 0, 0, 0});
        for (int32_t tile : {4096, 8192, 16384})
            for (int32_t sp : {10, 25, 50}) cand.push_back(dnatok_tuning{tile, 0, 0, 0, sp, 0});
        if (padded) {  // row bands, staged through LDS stages of 4 to 64 KiB; persistent ones of 4 and 8 KiB
            // (a 16 KiB persistent stage holds no band of 16 KiB, so it would run as row bands)
            for (int32_t tile : {4096, 8192, 16384, 32768, 65536}) cand.push_back(dnatok_tuning{tile, 0, 0, 0, 0, 1});
            for (int32_t tile : {4096, 8192}) cand.push_back(dnatok_tuning{tile, 0, 0, 0, 0, 3});
        }
    }
    const dnatok_tuning saved = load(v);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    DNATOK_HIP(hipEventCreate(&e0));
    DNATOK_HIP(hipEventCreate(&e1));
    int rc = DNATOK_OK;
    // one sample: kBatch back-to-back launches between one event pair (after
    // the previous sample has finished), the time per launch. Timing single
    // launches added an event's release and timestamp (about 18 us) to each,
    // whose noise could hide a 10% difference between candidates.
    constexpr int kBatch = 4;
    auto time_one = [&](float *ms) {
        if (hipEventRecord(e0, st) != hipSuccess) return set_error(DNATOK_EDEVICE, "hipEventRecord failed");
        for (int b = 0; b < kBatch; ++b) {
            int r = run();
            if (r != DNATOK_OK) return r;
        }
        if (hipEventRecord(e1, st) != hipSuccess) return set_error(DNATOK_EDEVICE, "hipEventRecord failed");
        if (hipEventSynchronize(e1) != hipSuccess) return set_error(DNATOK_EDEVICE, "hipEventSynchronize failed");
        if (hipEventElapsedTime(ms, e0, e1) != hipSuccess) return set_error(DNATOK_EDEVICE, "hipEventElapsedTime failed");
        *ms /= (float)kBatch;
        return DNATOK_OK;
    };
    auto median = [](std::vector<float> &ts) {
        std::nth_element(ts.begin(), ts.begin() + ts.size() / 2, ts.end());
        return ts[ts.size() / 2];
    };
    // Screen: every candidate, one warm-up sample and reps timed ones.
    std::vector<float> med(cand.size(), 0.0f);
    for (size_t ci = 0; ci < cand.size() && rc == DNATOK_OK; ++ci) {
        store(v, cand[ci]);
        std::vector<float> ts;
        for (int r = 0; r <= reps && rc == DNATOK_OK; ++r) {
            float ms = 0.0f;
            rc = time_one(&ms);
            if (r > 0) ts.push_back(ms);  // the first sample warms up
        }
        if (rc == DNATOK_OK) med[ci] = median(ts);
    }
    // Final: the three best of the screen again, 3 * reps launches each,
    // interleaved so that drift of the clocks or the neighbours' load hits
    // them alike; the smallest median wins.
    float best_t = -1.0f;
    dnatok_tuning best_c = saved;
    if (rc == DNATOK_OK && !cand.empty()) {
        std::vector<size_t> order(cand.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = i;
        const size_t nf = std::min<size_t>(3, order.size());
        std::partial_sort(order.begin(), order.begin() + nf, order.end(),
                          [&](size_t x, size_t y) { return med[x] < med[y]; });
        std::vector<std::vector<float>> ts(nf);
        for (int r = 0; r < 3 * reps && rc == DNATOK_OK; ++r)
            for (size_t f = 0; f < nf && rc == DNATOK_OK; ++f) {
                store(v, cand[order[f]]);
                float ms = 0.0f;
                rc = time_one(&ms);
                ts[f].push_back(ms);
            }
        for (size_t f = 0; f < nf && rc == DNATOK_OK; ++f) {
            const float m = median(ts[f]);
            if (best_t < 0.0f || m < best_t) {
                best_t = m;
                best_c = cand[order[f]];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != DNATOK_OK) {
        store(v, saved);
        return rc;
    }
    store(v, best_c);
    if (best) *best = best_c;
    if (best_ms) *best_ms = best_t;
    return DNATOK_OK;
}

}  // namespace

extern "C" {

int dnatok_autotune(dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets, int32_t n,
                    int32_t *d_ids, int64_t ids_capacity, int64_t *d_out_offsets, int8_t *d_mask,
                    const dnatok_encode_opts *opts, void *stream, int32_t reps, dnatok_tuning *best,
                    float *best_ms) {
    const bool padded = opts && opts->layout == DNATOK_PADDED;
    return autotune_loop(v, static_cast<hipStream_t>(stream), reps, padded, [&] {
        return dnatok_encode(v, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets, d_mask, opts,
                             stream);
    }, best, best_ms);
}

int dnatok_autotune_multi(dnatok_vocab *const *vocabs, int32_t n_vocabs, const uint8_t *d_bytes, int64_t nbytes,
                          const int64_t *d_offsets, int32_t n, int32_t *const *d_ids, const int64_t *ids_capacity,
                          int64_t *const *d_out_offsets, int8_t *const *d_mask, const dnatok_encode_opts *opts,
                          void *stream, int32_t reps, dnatok_tuning *best, float *best_ms) {
    if (!vocabs || n_vocabs < 1) return set_error(DNATOK_EINVAL, "no vocabularies");
    const bool padded = opts && opts[0].layout == DNATOK_PADDED;
    return autotune_loop(vocabs[0], static_cast<hipStream_t>(stream), reps, padded, [&] {
        return dnatok_encode_multi(vocabs, n_vocabs, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity,
                                   d_out_offsets, d_mask, opts, stream);
    }, best, best_ms);
}

int dnatok_graph_create(const dnatok_encode_call *calls, int32_t n_calls, dnatok_graph **out) {
    if (!out || (!calls && n_calls > 0)) return set_error(DNATOK_EINVAL, "null argument");
    if (n_calls < 1 || n_calls > 1024) return set_error(DNATOK_EINVAL, "n_calls must be 1..1024");
    *out = nullptr;
    auto g = new dnatok_graph();
    auto fail = [&](int rc) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        if (g->stream) {
            (void)hipStreamSynchronize(g->stream);
            drop_workspace(g->stream);
            (void)hipStreamDestroy(g->stream);
        }
        delete g;
        return rc;
    };
    auto run = [&](const dnatok_encode_call &c) {
        return dnatok_encode(c.v, c.d_bytes, c.nbytes, c.d_offsets, c.n, c.d_ids, c.ids_capacity, c.d_out_offsets,
                             c.d_mask, &c.opts, g->stream);
    };
    if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess)
        return fail(set_error(DNATOK_EDEVICE, "hipStreamCreateWithFlags failed"));
    // eager run: validates the calls and sizes the workspace the graph will use
    for (int32_t i = 0; i < n_calls; ++i) {
        const int rc = run(calls[i]);
        if (rc) return fail(rc);
    }
    if (hipStreamSynchronize(g->stream) != hipSuccess)
        return fail(set_error(DNATOK_EDEVICE, "hipStreamSynchronize failed"));
    if (hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(set_error(DNATOK_EDEVICE, "hipStreamBeginCapture failed"));
    int rc = DNATOK_OK;
    for (int32_t i = 0; i < n_calls && rc == DNATOK_OK; ++i) rc = run(calls[i]);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(g->stream, &graph);
    g->graph = graph;
    if (rc) return fail(rc);
    if (ec != hipSuccess || !graph) return fail(set_error(DNATOK_EDEVICE, "hipStreamEndCapture failed"));
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
        return fail(set_error(DNATOK_EDEVICE, "hipGraphInstantiate failed"));
    *out = g;
    return DNATOK_OK;
}

int dnatok_graph_launch(dnatok_graph *g, void *stream) {
    if (!g || !g->exec) return set_error(DNATOK_EINVAL, "null graph");
    DNATOK_HIP(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return DNATOK_OK;
}

int dnatok_graph_destroy(dnatok_graph *g) {
    if (!g) return DNATOK_OK;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    (void)hipDeviceSynchronize();  // replays on other streams may still read the workspace
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->stream) {
        drop_workspace(g->stream);
        (void)hipStreamDestroy(g->stream);
    }
    delete g;
    return DNATOK_OK;
}

}  // extern "C"
