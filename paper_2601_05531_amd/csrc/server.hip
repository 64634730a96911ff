// Serving loop: continuous batching of tokenize requests on one device.
//
// Paper: online serving puts tokenization on the latency path of each
// request (Discussion, "When Does DNATok Matter?"; the latency-bound
// real-model scenario of the Results), and the paper guards device memory
// with an out-of-memory retry (Design, "Robustness and compatibility"). Here
// admission is explicit: a request enters a batch only once the arena holds
// its input and output, and the arena is sized by the caller's budget.
//
// One worker thread owns the schedule:
//  1. finished batches (event query) hand their results back and free their
//     input region;
//  2. for every free stream slot, the oldest waiting request fixes the
//     vocabulary and specials flag of the next batch; waiting requests with
//     the same pair join it, in arrival order, up to max_batch requests /
//     max_batch_bytes, as far as the arena has room (the oldest request is
//     never overtaken by a smaller one of its kind);
//  3. the batch's bytes go to the device (pinned inputs directly, pageable
//     ones through the slot's pinned staging), one dnatok_encode runs on the
//     slot's stream and the output offsets come back to pinned host memory.
// Batches on different streams overlap on the device.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "hostbook.hpp"

namespace dnatok {
namespace {

constexpr int64_t kAlign = 256;
inline int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    const dnatok_vocab *vocab = nullptr;
    const uint8_t *h = nullptr;  // pinned caller memory, or own.data()
    std::vector<uint8_t> own;    // copy of a pageable input
    bool pinned = false;
    int64_t nbytes = 0;
    int32_t cls = 0;
    int64_t cap = 0;  // upper bound of its token count
    bool done = false;
    dnatok_request_result res{};
    int64_t batch = -1;
};

struct Batch {
    int64_t id = 0;
    int slot = -1;
    std::vector<uint64_t> tickets;
    int64_t in_off = -1, in_size = 0;    // bytes + offsets + out offsets
    int64_t out_off = -1, out_size = 0;  // ids
    int refs = 0;                        // results not yet released
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint8_t *staging = nullptr;   // pinned
    int64_t *h_offs = nullptr;    // pinned [max_batch + 1]: input offsets
    int64_t *h_oofs = nullptr;    // pinned [max_batch + 1]: output offsets read back
    int64_t batch = -1;           // in flight, or -1
};

}  // namespace
}  // namespace dnatok

struct dnatok_server {
    dnatok_server_opts o{};
    int device = 0;
    uint8_t *d_arena = nullptr;
    dnatok::Arena arena;
    std::vector<dnatok::Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, dnatok::Request> reqs;
    std::unordered_map<int64_t, dnatok::Batch> batches;
    uint64_t next_ticket = 1;
    int64_t next_batch = 1;
    int64_t n_done = 0, n_batches = 0;
    bool stopping = false;
    std::thread worker;
    dnatok::Clock::time_point t0;
    int64_t arena_bytes = 0;
};

namespace dnatok {
namespace {

double now_s(const dnatok_server *s) {
    return std::chrono::duration<double>(Clock::now() - s->t0).count();
}

int64_t token_cap(const dnatok_vocab *v, int64_t L, int32_t cls) {
    const int64_t k = (v->kind == DNATOK_KMER) ? v->k : 1;
    return (L + k - 1) / k + 2 * (int64_t)cls;
}

// Device bytes of a batch's two regions.
void batch_sizes(int64_t in_bytes, int64_t n, int64_t cap, int64_t *in_size, int64_t *out_size) {
    *in_size = align_up(in_bytes) + 2 * align_up(8 * (n + 1));
    *out_size = align_up(4 * std::max<int64_t>(cap, 1));
}

void fail_request(dnatok_server *s, Request &r, int status) {
    r.done = true;
    r.res = dnatok_request_result{};
    r.res.status = status;
    r.res.t_submit = r.res.t_start = r.res.t_done = now_s(s);
    ++s->n_done;
}

// Completion of the batch in slot `si` (called with the lock held).
void complete(dnatok_server *s, int si) {
    Slot &sl = s->slots[si];
    Batch &b = s->batches[sl.batch];
    uint32_t flags = 0;
    hipStream_t st = sl.stream;
    if (dnatok_sync_status(st, &flags) != DNATOK_OK) flags = DNATOK_DERR_INTERNAL;
    const double t = now_s(s);
    const int32_t *ids = reinterpret_cast<const int32_t *>(s->d_arena + b.out_off);
    for (size_t i = 0; i < b.tickets.size(); ++i) {
        Request &r = s->reqs[b.tickets[i]];
        r.done = true;
        r.res.d_ids = ids + sl.h_oofs[i];
        r.res.n_tokens = sl.h_oofs[i + 1] - sl.h_oofs[i];
        r.res.status = DNATOK_OK;
        r.res.dev_flags = flags;
        r.res.t_done = t;
        r.h = nullptr;
        r.own.clear();
        r.own.shrink_to_fit();
        ++s->n_done;
    }
    s->arena.release(b.in_off, b.in_size);
    b.in_off = -1;
    sl.batch = -1;
}

// Forms and launches one batch on slot `si` (lock held). Returns true when a
// batch was launched.
bool launch(dnatok_server *s, int si) {
    if (s->pending.empty()) return false;
    Slot &sl = s->slots[si];
    const Request &head = s->reqs[s->pending.front()];
    const dnatok_vocab *v = head.vocab;
    const int32_t cls = head.cls;
    // candidates in arrival order
    std::vector<uint64_t> pick;
    int64_t bytes = 0, cap = 0;
    for (uint64_t t : s->pending) {
        const Request &r = s->reqs[t];
        if (r.vocab != v || r.cls != cls) continue;
        if (!pick.empty() && ((int32_t)pick.size() >= s->o.max_batch || bytes + r.nbytes > s->o.max_batch_bytes))
            break;
        pick.push_back(t);
        bytes += r.nbytes;
        cap += r.cap;
    }
    // as many of them as the arena holds (at least the oldest, or nothing)
    int64_t in_off = -1, out_off = -1, in_size = 0, out_size = 0;
    while (!pick.empty()) {
        batch_sizes(bytes, (int64_t)pick.size(), cap, &in_size, &out_size);
        in_off = s->arena.alloc(in_size);
        if (in_off >= 0) {
            out_off = s->arena.alloc(out_size);
            if (out_off >= 0) break;
            s->arena.release(in_off, in_size);
            in_off = -1;
        }
        const Request &last = s->reqs[pick.back()];
        bytes -= last.nbytes;
        cap -= last.cap;
        pick.pop_back();
    }
    if (pick.empty()) return false;  // wait for memory: the oldest request keeps its place

    const int64_t id = s->next_batch++;
    Batch &b = s->batches[id];
    b.id = id;
    b.slot = si;
    b.tickets = pick;
    b.in_off = in_off;
    b.in_size = in_size;
    b.out_off = out_off;
    b.out_size = out_size;
    b.refs = (int)pick.size();
    {
        std::deque<uint64_t> rest;
        size_t j = 0;
        for (uint64_t t : s->pending) {
            if (j < pick.size() && t == pick[j]) {
                ++j;
                continue;
            }
            rest.push_back(t);
        }
        s->pending.swap(rest);
    }
    const int n = (int)pick.size();
    uint8_t *d_in = s->d_arena + in_off;
    int64_t *d_offs = reinterpret_cast<int64_t *>(d_in + align_up(bytes));
    int64_t *d_oofs = reinterpret_cast<int64_t *>(reinterpret_cast<uint8_t *>(d_offs) + align_up(8 * (n + 1)));
    int32_t *d_ids = reinterpret_cast<int32_t *>(s->d_arena + out_off);
    const double t = now_s(s);
    int64_t pos = 0, staged = 0;
    sl.h_offs[0] = 0;
    int rc = DNATOK_OK;
    for (int i = 0; i < n; ++i) {
        Request &r = s->reqs[pick[i]];
        r.batch = id;
        r.res.t_start = t;
        if (r.nbytes > 0) {
            if (r.pinned) {
                if (hipMemcpyAsync(d_in + pos, r.h, (size_t)r.nbytes, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
                    rc = DNATOK_EDEVICE;
            } else {
                std::memcpy(sl.staging + staged, r.h, (size_t)r.nbytes);
                if (hipMemcpyAsync(d_in + pos, sl.staging + staged, (size_t)r.nbytes, hipMemcpyHostToDevice,
                                   sl.stream) != hipSuccess)
                    rc = DNATOK_EDEVICE;
                staged += r.nbytes;
            }
        }
        pos += r.nbytes;
        sl.h_offs[i + 1] = pos;
    }
    if (hipMemcpyAsync(d_offs, sl.h_offs, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice, sl.stream) !=
        hipSuccess)
        rc = DNATOK_EDEVICE;
    dnatok_encode_opts eo{};
    eo.add_cls_sep = cls;
    eo.layout = DNATOK_PACKED;
    if (rc == DNATOK_OK)
        rc = dnatok_encode(v, d_in, bytes, d_offs, n, d_ids, out_size / 4, d_oofs, nullptr, &eo, sl.stream);
    if (rc == DNATOK_OK &&
        hipMemcpyAsync(sl.h_oofs, d_oofs, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDeviceToHost, sl.stream) !=
            hipSuccess)
        rc = DNATOK_EDEVICE;
    if (rc == DNATOK_OK && hipEventRecord(sl.done, sl.stream) != hipSuccess) rc = DNATOK_EDEVICE;
    ++s->n_batches;
    if (rc != DNATOK_OK) {
        // the batch failed before reaching the device: fail its requests
        (void)hipStreamSynchronize(sl.stream);
        for (uint64_t tk : pick) fail_request(s, s->reqs[tk], rc);
        s->arena.release(in_off, in_size);
        s->arena.release(out_off, out_size);
        s->batches.erase(id);
        for (uint64_t tk : pick) s->reqs[tk].batch = -1;
        s->cv_done.notify_all();
        return true;
    }
    // the output offsets are relative to the batch's ids
    sl.batch = id;
    return true;
}

void worker_main(dnatok_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progress = false;
        bool inflight = false;
        for (int i = 0; i < (int)s->slots.size(); ++i) {
            Slot &sl = s->slots[i];
            if (sl.batch < 0) continue;
            if (hipEventQuery(sl.done) == hipSuccess) {
                complete(s, i);
                progress = true;
            } else {
                inflight = true;
            }
        }
        if (progress) s->cv_done.notify_all();
        for (int i = 0; i < (int)s->slots.size(); ++i) {
            if (s->slots[i].batch >= 0) continue;
            if (!launch(s, i)) break;
            inflight = true;
            progress = true;
        }
        if (s->stopping && !inflight) {
            // nothing runs and nothing more fits: what is still waiting fails
            for (uint64_t t : s->pending) fail_request(s, s->reqs[t], DNATOK_ESTATE);
            s->pending.clear();
            s->cv_done.notify_all();
            break;
        }
        if (!progress) {
            // batches in flight: poll soon; idle: sleep until a submission
            if (inflight)
                s->cv_work.wait_for(lk, std::chrono::microseconds(20));
            else
                s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

}  // namespace
}  // namespace dnatok

using namespace dnatok;

extern "C" {

int dnatok_server_create(const dnatok_server_opts *opts, dnatok_server **out) {
    if (!opts || !out) return set_error(DNATOK_EINVAL, "null argument");
    *out = nullptr;
    dnatok_server_opts o = *opts;
    if (o.n_streams < 1 || o.n_streams > 16) return set_error(DNATOK_EINVAL, "n_streams must be 1..16");
    if (o.max_batch < 1) return set_error(DNATOK_EINVAL, "max_batch must be >= 1");
    if (o.max_batch_bytes < 1) return set_error(DNATOK_EINVAL, "max_batch_bytes must be >= 1");
    if (o.staging_bytes < o.max_batch_bytes) return set_error(DNATOK_EINVAL, "staging_bytes < max_batch_bytes");
    // per stream: BPE scratch and scan workspace for the largest batch
    // (sized for the smallest BPE item length a vocabulary may be tuned to)
    const int64_t scratch = bpe_scratch_bytes(o.max_batch_bytes, o.max_batch, kBpeItemBytesMin);
    const int64_t tiles = bpe_workspace_tiles(o.max_batch_bytes, o.max_batch, kBpeItemBytesMin);
    const int64_t ws_bytes = 256 + 2 * 8 * std::max<int64_t>(tiles, 4096);
    const int64_t reserve = (int64_t)o.n_streams * (scratch + ws_bytes);
    const int64_t arena = (o.budget_bytes - reserve) / kAlign * kAlign;
    int64_t in_size = 0, out_size = 0;
    batch_sizes(o.max_batch_bytes, 1, o.max_batch_bytes + 2, &in_size, &out_size);
    if (arena < in_size + out_size)
        return set_error(DNATOK_EINVAL, "budget %lld leaves no arena for one batch after %lld bytes of per-stream "
                         "scratch", (long long)o.budget_bytes, (long long)reserve);
    auto s = std::make_unique<dnatok_server>();
    s->o = o;
    s->t0 = Clock::now();
    DNATOK_HIP(hipGetDevice(&s->device));
    void *p = nullptr;
    DNATOK_HIP(dev_alloc(&p, (size_t)arena));
    s->d_arena = static_cast<uint8_t *>(p);
    s->arena_bytes = arena;
    s->arena.reset(arena);
    s->slots.resize(o.n_streams);
    auto cleanup = [&](int rc) {
        for (Slot &sl : s->slots) {
            if (sl.stream) {
                drop_workspace(sl.stream);
                (void)hipStreamDestroy(sl.stream);
            }
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.staging) (void)hipHostFree(sl.staging);
            if (sl.h_offs) (void)hipHostFree(sl.h_offs);
            if (sl.h_oofs) (void)hipHostFree(sl.h_oofs);
        }
        (void)hipFree(s->d_arena);
        return rc;
    };
    for (Slot &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
            return cleanup(set_error(DNATOK_EDEVICE, "stream/event creation failed"));
        if (host_alloc(&p, (size_t)o.staging_bytes) != hipSuccess)
            return cleanup(set_error(DNATOK_ENOMEM, "pinned staging (%lld bytes)", (long long)o.staging_bytes));
        sl.staging = static_cast<uint8_t *>(p);
        if (host_alloc(&p, sizeof(int64_t) * (size_t)(o.max_batch + 1)) != hipSuccess)
            return cleanup(set_error(DNATOK_ENOMEM, "pinned offsets"));
        sl.h_offs = static_cast<int64_t *>(p);
        if (host_alloc(&p, sizeof(int64_t) * (size_t)(o.max_batch + 1)) != hipSuccess)
            return cleanup(set_error(DNATOK_ENOMEM, "pinned offsets"));
        sl.h_oofs = static_cast<int64_t *>(p);
        // grow the stream's workspace now so no batch allocates on the hot path
        Workspace *ws = nullptr;
        int rc = get_workspace(sl.stream, tiles, &ws);
        if (rc == DNATOK_OK) rc = ensure_scratch(ws, scratch);
        if (rc != DNATOK_OK) return cleanup(rc);
    }
    dnatok_server *raw = s.release();
    raw->worker = std::thread(worker_main, raw);
    *out = raw;
    return DNATOK_OK;
}

int dnatok_server_submit(dnatok_server *s, const dnatok_vocab *v, const uint8_t *h_bytes, int64_t nbytes,
                         int32_t add_cls_sep, uint64_t *ticket) {
    if (!s || !v || !ticket) return set_error(DNATOK_EINVAL, "null argument");
    if (nbytes < 0 || (nbytes > 0 && !h_bytes)) return set_error(DNATOK_EINVAL, "bad input");
    if (v->device != s->device) return set_error(DNATOK_EINVAL, "vocabulary and server are on different devices");
    if (nbytes > s->o.max_batch_bytes)
        return set_error(DNATOK_EBUDGET, "request of %lld bytes exceeds max_batch_bytes", (long long)nbytes);
    const int32_t cls = add_cls_sep ? 1 : 0;
    const int64_t cap = token_cap(v, nbytes, cls);
    int64_t in_size = 0, out_size = 0;
    batch_sizes(nbytes, 1, cap, &in_size, &out_size);
    if (in_size + out_size > s->arena_bytes)
        return set_error(DNATOK_EBUDGET, "request needs %lld arena bytes, the arena has %lld",
                         (long long)(in_size + out_size), (long long)s->arena_bytes);
    Request r;
    r.vocab = v;
    r.nbytes = nbytes;
    r.cls = cls;
    r.cap = cap;
    if (nbytes > 0) {
        hipPointerAttribute_t attr;
        const bool pinned = hipPointerGetAttributes(&attr, h_bytes) == hipSuccess && attr.type == hipMemoryTypeHost;
        (void)hipGetLastError();  // a pageable pointer leaves an error behind
        r.pinned = pinned;
        if (pinned) {
            r.h = h_bytes;
        } else {
            r.own.assign(h_bytes, h_bytes + nbytes);
            r.h = r.own.data();
        }
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return set_error(DNATOK_ESTATE, "server is shutting down");
        r.ticket = s->next_ticket++;
        r.res.t_submit = now_s(s);
        *ticket = r.ticket;
        s->pending.push_back(r.ticket);
        s->reqs.emplace(r.ticket, std::move(r));
    }
    s->cv_work.notify_one();
    return DNATOK_OK;
}

int dnatok_server_poll(dnatok_server *s, uint64_t ticket, dnatok_request_result *out) {
    if (!s || !out) return set_error(DNATOK_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(DNATOK_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second.done) return 1;
    *out = it->second.res;
    return DNATOK_OK;
}

int dnatok_server_wait(dnatok_server *s, uint64_t ticket, dnatok_request_result *out) {
    if (!s || !out) return set_error(DNATOK_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(DNATOK_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    // A submission made while this thread waits may rehash the map, which
    // invalidates iterators but never references to its elements.
    const Request &r = it->second;
    s->cv_done.wait(lk, [&] { return r.done; });
    *out = r.res;
    return DNATOK_OK;
}

int dnatok_server_release(dnatok_server *s, uint64_t ticket) {
    if (!s) return set_error(DNATOK_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(DNATOK_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second.done) return set_error(DNATOK_ESTATE, "request %llu is not done", (unsigned long long)ticket);
    const int64_t bid = it->second.batch;
    s->reqs.erase(it);
    if (bid >= 0) {
        auto bt = s->batches.find(bid);
        if (bt != s->batches.end() && --bt->second.refs == 0) {
            s->arena.release(bt->second.out_off, bt->second.out_size);
            s->batches.erase(bt);
        }
    }
    s->cv_work.notify_one();
    return DNATOK_OK;
}

double dnatok_server_now(const dnatok_server *s) { return s ? now_s(s) : 0.0; }

int dnatok_server_stats(const dnatok_server *s, int64_t *requests, int64_t *batches, int64_t *peak_bytes) {
    if (!s) return set_error(DNATOK_EINVAL, "null server");
    auto *m = const_cast<dnatok_server *>(s);
    std::lock_guard<std::mutex> lk(m->mu);
    if (requests) *requests = s->n_done;
    if (batches) *batches = s->n_batches;
    if (peak_bytes) *peak_bytes = s->arena.peak();
    return DNATOK_OK;
}

int dnatok_server_destroy(dnatok_server *s) {
    if (!s) return DNATOK_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (Slot &sl : s->slots) {
        if (sl.stream) {
            (void)hipStreamSynchronize(sl.stream);
            drop_workspace(sl.stream);
            (void)hipStreamDestroy(sl.stream);
        }
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.staging) (void)hipHostFree(sl.staging);
        if (sl.h_offs) (void)hipHostFree(sl.h_offs);
        if (sl.h_oofs) (void)hipHostFree(sl.h_oofs);
    }
    if (s->d_arena) (void)hipFree(s->d_arena);
    delete s;
    return DNATOK_OK;
}

}  // extern "C"
