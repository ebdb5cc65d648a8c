// Request loop with continuous batching (the serving layer around the batched engine).
//
// A worker thread owns the device side.  Each pass it
//   1. retires finished launch groups (their completion events have fired): marks their
//      requests done, returns their budget and slots, frees their workspace;
//   2. admits queued requests in arrival order while the HBM ray-state budget and the slot
//      limit allow (a request never jumps ahead of an earlier one);
//   3. launches the newly admitted requests together as one engine batch on the next of its
//      streams, with an event behind it.
// Requests that arrive while others run are therefore admitted as soon as budget and slots
// free up, and their work overlaps on the device with the groups still in flight.  In the
// plain mode (the baseline) one request at a time goes through hcc_encode, hcc_sort and
// hcc_trace and the next starts only after it finished.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hcc_internal.h"

namespace hcc {
size_t batch_table_bytes(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits);
hcc_status batch_workspace(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits, size_t* bytes);
hcc_status engine_workspace(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits, size_t* bytes);
hcc_status batch_check(const void* d_ws, hipStream_t stream, uint32_t* ok);
hcc_status batch_launch(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits,
                        const hcc_batch_opts& o, void* d_ws, size_t ws_bytes, hipStream_t stream, void* pinned,
                        size_t pinned_bytes);
size_t graph_table_bytes(uint32_t max_batches);
hcc_status graph_capture(uint32_t max_batches, uint32_t key_bits, const hcc_batch_opts& o, void* pinned,
                         void* d_tables, hipStream_t capture_stream, hipGraphExec_t* exec);
hcc_status graph_launch(const hcc_batch_desc* d, uint32_t nb, uint32_t mode, uint32_t key_bits,
                        const hcc_batch_opts& o, void* d_ws, size_t ws_bytes, uint32_t max_batches, void* pinned,
                        void* d_tables, hipGraphExec_t exec, hipStream_t stream);
hcc_status encode_hcc(const hcc_cut_s* cut, uint32_t key_bits, const hcc_ray* d_rays, uint32_t n, void* d_keys,
                      hipStream_t stream);
hcc_status encode_twopoint(const hcc_bvh_s* bvh, uint32_t key_bits, const hcc_ray* d_rays, uint32_t n,
                           void* d_keys, hipStream_t stream);
hcc_status trace(const hcc_bvh_s* b, const hcc_ray* rays, const uint32_t* perm, uint32_t n, bool closest,
                 hcc_hit* hits, uint8_t* occ, const hcc_trace_opts& o, hipStream_t s);
}  // namespace hcc

using Clock = std::chrono::steady_clock;

namespace {

enum : uint32_t { kQueued = 0, kRunning = 1, kDone = 2, kCancelled = 3, kFailed = 4 };

struct Req {
    hcc_batch_desc desc{};
    size_t bytes = 0;
    uint32_t state = kQueued;
    Clock::time_point t_submit, t_start, t_done;
};

// A captured launch graph with its staging and device table buffers (graph mode).
struct Slot {
    void* pinned = nullptr;
    void* d_tables = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct Group {
    std::vector<uint64_t> ids;
    int slot = -1;
    void* direct[3] = {nullptr, nullptr, nullptr};   // a large request's own keys / perm / sort workspace
    hipEvent_t done = nullptr;
    void* ws = nullptr;
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
};

}  // namespace

struct hcc_server_s {
    hcc_server_opts opts{};
    int device = 0;
    std::vector<hipStream_t> streams;
    size_t next_stream = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, Req> reqs;
    std::vector<Group> inflight;
    // reused between groups: pinned staging buffers for the launch tables (size, pointer)
    // and completion events; allocating either per launch costs more than a small launch
    std::vector<std::pair<size_t, void*>> pinned_free;
    std::vector<hipEvent_t> events_free;
    std::vector<Slot> slots;        // graph mode: every slot ever made
    std::vector<int> slots_free;
    hcc::Allocator alloc;           // hooks at creation; without hooks, stream-ordered hipMallocAsync
    uint64_t next_id = 1;
    size_t used_bytes = 0;
    uint32_t running = 0;
    uint64_t launches = 0, completed = 0;
    std::string error;
    bool stop = false;
    std::thread worker;
    uint64_t magic = 0x6863637372760001ull;
};

namespace {

bool valid_server(const hcc_server_s* s) { return s && s->magic == 0x6863637372760001ull; }

// Device bytes a request holds while admitted: its rays and results, plus the engine's
// per-ray workspace (keys, permutation, ping-pong buffers) of a batch of that size.
size_t request_bytes(const hcc_batch_desc& d, uint32_t mode, uint32_t key_bits) {
    size_t ws = 0;
    hcc::batch_workspace(&d, 1, mode, key_bits, &ws);
    return (size_t)d.n * (sizeof(hcc_ray) + (d.mode == HCC_TRACE_CLOSEST ? sizeof(hcc_hit) : 1)) + ws;
}

void* dev_get(hcc_server_s* s, size_t bytes, hipStream_t st) {
    if (s->alloc.alloc) return s->alloc.get(bytes, st);
    void* p = nullptr;
    if (hipMallocAsync(&p, bytes, st) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void dev_put(hcc_server_s* s, void* p, hipStream_t st) {
    if (!p) return;
    if (s->alloc.alloc) s->alloc.put(p, st);
    else (void)hipFreeAsync(p, st);
}

void finish_group(hcc_server_s* s, Group& g, bool ok) {
    const auto now = Clock::now();
    for (uint64_t id : g.ids) {
        Req& r = s->reqs[id];
        r.state = ok ? kDone : kFailed;
        r.t_done = now;
        s->used_bytes -= r.bytes;
        s->running -= 1;
        s->completed += 1;
    }
    if (g.ws) dev_put(s, g.ws, g.stream);
    for (void* b : g.direct) dev_put(s, b, g.stream);
    if (g.pinned) s->pinned_free.emplace_back(g.pinned_bytes, g.pinned);
    if (g.done) s->events_free.push_back(g.done);
    if (g.slot >= 0) s->slots_free.push_back(g.slot);
    g = Group();
}

// A pinned buffer of at least `bytes` from the free list (the smallest that fits), else a new one.
void* take_pinned(hcc_server_s* s, size_t bytes, size_t* got) {
    size_t best = s->pinned_free.size();
    for (size_t i = 0; i < s->pinned_free.size(); ++i)
        if (s->pinned_free[i].first >= bytes && (best == s->pinned_free.size() ||
                                                 s->pinned_free[i].first < s->pinned_free[best].first))
            best = i;
    if (best < s->pinned_free.size()) {
        void* p = s->pinned_free[best].second;
        *got = s->pinned_free[best].first;
        s->pinned_free.erase(s->pinned_free.begin() + (ptrdiff_t)best);
        return p;
    }
    const size_t sz = std::max<size_t>(bytes, 64u << 10);
    void* p = nullptr;
    if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) return nullptr;
    *got = sz;
    return p;
}

// A free graph slot, capturing a new one when none is free (-1 on failure).
int take_slot(hcc_server_s* s) {
    if (!s->slots_free.empty()) {
        const int i = s->slots_free.back();
        s->slots_free.pop_back();
        return i;
    }
    Slot sl;
    const size_t bytes = hcc::graph_table_bytes(s->opts.max_group);
    if (hipHostMalloc(&sl.pinned, bytes, hipHostMallocDefault) != hipSuccess) return -1;
    std::memset(sl.pinned, 0, bytes);
    sl.d_tables = s->alloc.get(bytes, s->streams[0]);
    hipStream_t cap = nullptr;
    bool ok = sl.d_tables && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hcc::graph_capture(s->opts.max_group, s->opts.key_bits, s->opts.batch, sl.pinned, sl.d_tables, cap,
                                  &sl.exec) == HCC_OK;
    if (cap) (void)hipStreamDestroy(cap);
    if (!ok) {
        if (sl.d_tables) s->alloc.put(sl.d_tables, s->streams[0]);
        (void)hipHostFree(sl.pinned);
        return -1;
    }
    s->slots.push_back(sl);
    return (int)s->slots.size() - 1;
}

hipEvent_t take_event(hcc_server_s* s) {
    if (!s->events_free.empty()) {
        hipEvent_t e = s->events_free.back();
        s->events_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// Plain mode: one request through encode / sort / trace, waited for before the next.
// One request through hcc_encode, hcc_sort and hcc_trace's kernels, enqueued on st; the
// buffers it takes (keys, permutation, sort workspace) are returned in bufs for the caller
// to release once the stream has passed them.
bool enqueue_direct(hcc_server_s* s, const hcc_batch_desc& d, hipStream_t st, void* bufs[3]) {
    const uint32_t mode = s->opts.key_mode, kb = s->opts.key_bits;
    bufs[0] = bufs[1] = bufs[2] = nullptr;
    bool ok = true;
    if (mode != HCC_KEY_NONE && d.n > 0) {
        const size_t ks = kb <= 32 ? 4 : 8;
        const size_t wsb = hcc::sort_workspace_bytes(d.n, kb);
        ok = (bufs[0] = dev_get(s, (size_t)d.n * ks, st)) != nullptr &&
             (bufs[1] = dev_get(s, (size_t)d.n * 4, st)) != nullptr && (bufs[2] = dev_get(s, wsb, st)) != nullptr;
        if (ok) ok = (mode == HCC_KEY_HCC ? hcc::encode_hcc(d.cut, kb, d.d_rays, d.n, bufs[0], st)
                                          : hcc::encode_twopoint(d.bvh, kb, d.d_rays, d.n, bufs[0], st)) == HCC_OK;
        if (ok) ok = hcc::radix_sort(bufs[0], kb, d.n, (uint32_t*)bufs[1], nullptr, nullptr, bufs[2], wsb, st) == HCC_OK;
    }
    hcc_trace_opts to{};   // the full-device trace: persistent 4-wide traversal (quantised nodes where
                           // the BVH has them), LDS short stack
    to.persistent = 1;
    to.stack = HCC_STACK_SHORT;
    to.refill = 32;
    to.chunk = 64;
    to.flags = HCC_TRACE_WIDE | (d.bvh->quant_ok ? HCC_TRACE_QUANT : 0u);
    if (ok && d.n > 0)
        ok = hcc::trace(d.bvh, d.d_rays, (const uint32_t*)bufs[1], d.n, d.mode == HCC_TRACE_CLOSEST, d.d_hits,
                        d.d_occluded, to, st) == HCC_OK;
    return ok;
}

// Plain mode: one request, waited for before the next.
bool run_plain(hcc_server_s* s, const hcc_batch_desc& d) {
    hipStream_t st = s->streams[0];
    void* bufs[3];
    const bool ok = enqueue_direct(s, d, st, bufs);
    const bool synced = hipStreamSynchronize(st) == hipSuccess;
    for (void* b : bufs) dev_put(s, b, st);
    return synced && ok;
}

void worker_loop(hcc_server_s* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        // 1. retire finished groups
        for (auto& g : s->inflight) {
            if (!g.done) continue;
            const hipError_t q = hipEventQuery(g.done);
            if (q == hipSuccess) {
                uint32_t ok = 1;
                if (g.ws && hcc::batch_check(g.ws, g.stream, &ok) == HCC_OK && !ok)
                    s->error = "an engine launch gave up waiting on a dependency";
                finish_group(s, g, ok != 0);
            }
            else if (q != hipErrorNotReady) finish_group(s, g, false);
        }
        s->inflight.erase(std::remove_if(s->inflight.begin(), s->inflight.end(),
                                         [](const Group& g) { return g.ids.empty(); }),
                          s->inflight.end());
        if (s->stop && s->pending.empty() && s->inflight.empty()) break;

        // 2. admission in arrival order
        std::vector<uint64_t> admit;
        while (!s->pending.empty()) {
            const uint64_t id = s->pending.front();
            Req& r = s->reqs[id];
            if (r.state == kCancelled) {
                s->pending.pop_front();
                continue;
            }
            const bool slots = s->running + admit.size() < s->opts.max_inflight;
            const bool budget = s->used_bytes + r.bytes <= s->opts.budget_bytes;
            const bool room = admit.size() < (s->opts.plain ? 1u : s->opts.max_group);
            if (!(slots && budget && room)) break;
            s->pending.pop_front();
            s->used_bytes += r.bytes;
            r.state = kRunning;
            r.t_start = Clock::now();
            admit.push_back(id);
        }
        s->running += (uint32_t)admit.size();

        // 3. launch
        if (!admit.empty()) {
            if (s->opts.plain) {
                const hcc_batch_desc d = s->reqs[admit[0]].desc;
                lk.unlock();
                const bool ok = run_plain(s, d);
                lk.lock();
                Group g;
                g.ids = admit;
                finish_group(s, g, ok);
                s->launches += 1;
                continue;
            }
            // large requests run through the full-device kernels, each on the next stream; the
            // rest go together into one engine launch
            // (a request admitted alone has nothing to share a launch with: it goes direct too)
            std::vector<uint64_t> small;
            size_t n_small = 0;
            for (uint64_t id : admit) n_small += s->reqs[id].desc.n < s->opts.direct_min ? 1 : 0;
            for (uint64_t id : admit) {
                if (s->reqs[id].desc.n < s->opts.direct_min && (n_small > 1 || s->opts.direct_min == 0xFFFFFFFFu)) {
                    small.push_back(id);
                    continue;
                }
                Group g;
                g.ids = {id};
                g.stream = s->streams[s->next_stream++ % s->streams.size()];
                bool ok = enqueue_direct(s, s->reqs[id].desc, g.stream, g.direct);
                ok = ok && (g.done = take_event(s)) != nullptr;
                ok = ok && hipEventRecord(g.done, g.stream) == hipSuccess;
                s->launches += 1;
                if (!ok) {
                    s->error = "launch failed: " + std::string(hcc_last_error());
                    (void)hipStreamSynchronize(g.stream);
                    finish_group(s, g, false);
                } else {
                    s->inflight.push_back(std::move(g));
                }
            }
            if (small.empty()) continue;
            std::vector<hcc_batch_desc> ds;
            for (uint64_t id : small) ds.push_back(s->reqs[id].desc);
            Group g;
            g.ids = small;
            g.stream = s->streams[s->next_stream++ % s->streams.size()];
            bool ok = hcc::engine_workspace(ds.data(), (uint32_t)ds.size(), s->opts.key_mode, s->opts.key_bits,
                                           &g.bytes) == HCC_OK;
            const size_t tb = hcc::batch_table_bytes(ds.data(), (uint32_t)ds.size(), s->opts.key_mode,
                                                     s->opts.key_bits);
            ok = ok && (g.ws = dev_get(s, g.bytes, g.stream)) != nullptr;
            if (s->opts.graphs) {
                ok = ok && (g.slot = take_slot(s)) >= 0;
                ok = ok && hcc::graph_launch(ds.data(), (uint32_t)ds.size(), s->opts.key_mode, s->opts.key_bits,
                                             s->opts.batch, g.ws, g.bytes, s->opts.max_group,
                                             s->slots[g.slot].pinned, s->slots[g.slot].d_tables,
                                             s->slots[g.slot].exec, g.stream) == HCC_OK;
            } else {
                ok = ok && (g.pinned = take_pinned(s, tb, &g.pinned_bytes)) != nullptr;
                ok = ok && hcc::batch_launch(ds.data(), (uint32_t)ds.size(), s->opts.key_mode, s->opts.key_bits,
                                             s->opts.batch, g.ws, g.bytes, g.stream, g.pinned, tb) == HCC_OK;
            }
            ok = ok && (g.done = take_event(s)) != nullptr;
            ok = ok && hipEventRecord(g.done, g.stream) == hipSuccess;
            s->launches += 1;
            if (!ok) {
                s->error = "launch failed: " + std::string(hcc_last_error());
                (void)hipStreamSynchronize(g.stream);   // nothing may still read the staging buffer
                finish_group(s, g, false);
            } else {
                s->inflight.push_back(std::move(g));
            }
            continue;
        }
        // 4. wait: poll quickly while work is on the device, sleep otherwise
        if (!s->inflight.empty()) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(10));
            lk.lock();
        } else {
            s->cv.wait_for(lk, std::chrono::milliseconds(2));
        }
    }
}

}  // namespace

using namespace hcc;

extern "C" {

__attribute__((visibility("default"))) hcc_status hcc_server_create(const hcc_server_opts* opts, hcc_server* out) {
    if (!out) return fail(HCC_ERR_INVALID, "hcc_server_create: null out");
    hcc_server_opts o{};
    if (opts) o = *opts;
    if (o.budget_bytes == 0) o.budget_bytes = 64ull << 30;
    if (o.max_inflight == 0) o.max_inflight = 64;
    if (o.max_group == 0) o.max_group = 16;
    if (o.direct_min == 0) o.direct_min = 65536;
    if (o.streams == 0) o.streams = 4;
    if (o.key_bits == 0) o.key_bits = 32;
    if (o.key_bits > 64 || o.streams > 32 || o.key_mode > HCC_KEY_TWOPOINT || (o.batch.flags & ~(HCC_TRACE_WIDE | HCC_TRACE_SLAB | HCC_TRACE_QUANT)) ||
        o.batch.stack > HCC_BATCH_STACK_SCRATCH)
        return fail(HCC_ERR_INVALID, "hcc_server_create: bad options");
    o.batch.direct_min = 0;   // large requests are routed by the server itself (direct_min above)
    hcc_server_s* s = new hcc_server_s();
    s->opts = o;
    s->alloc = hcc::current_allocator();
    (void)hipGetDevice(&s->device);
    for (uint32_t i = 0; i < o.streams; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return fail(HCC_ERR_DEVICE, "hcc_server_create: stream creation failed");
        }
        s->streams.push_back(st);
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return HCC_OK;
}

__attribute__((visibility("default"))) hcc_status hcc_server_submit(hcc_server s, const hcc_batch_desc* req,
                                                                    uint64_t* id) {
    if (!valid_server(s) || !req || !id) return fail(HCC_ERR_INVALID, "hcc_server_submit: invalid argument");
    const hcc_batch_desc& d = *req;
    if (!d.bvh || d.bvh->magic != 0x6863636276680001ull) return fail(HCC_ERR_INVALID, "hcc_server_submit: invalid bvh");
    if (s->opts.key_mode == HCC_KEY_HCC && (!d.cut || d.cut->magic != 0x6863636375740001ull || d.cut->bvh != d.bvh))
        return fail(HCC_ERR_INVALID, "hcc_server_submit: HCC needs a cut of the request's bvh");
    if (d.n >= (1u << 30) || (d.n > 0 && !d.d_rays) || (d.mode != HCC_TRACE_CLOSEST && d.mode != HCC_TRACE_ANY) ||
        (d.n > 0 && d.mode == HCC_TRACE_CLOSEST && !d.d_hits) || (d.n > 0 && d.mode == HCC_TRACE_ANY && !d.d_occluded))
        return fail(HCC_ERR_INVALID, "hcc_server_submit: bad request");
    const size_t bytes = request_bytes(d, s->opts.key_mode, s->opts.key_bits);
    if (bytes > s->opts.budget_bytes)
        return fail(HCC_ERR_BUDGET, "hcc_server_submit: request needs " + std::to_string(bytes) +
                                        " bytes, more than the whole budget");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(HCC_ERR_INVALID, "hcc_server_submit: server is shutting down");
    const uint64_t rid = s->next_id++;
    Req& r = s->reqs[rid];
    r.desc = d;
    r.bytes = bytes;
    r.t_submit = Clock::now();
    s->pending.push_back(rid);
    s->cv.notify_one();
    *id = rid;
    return HCC_OK;
}

__attribute__((visibility("default"))) hcc_status hcc_server_poll(hcc_server s, uint64_t id, uint32_t* state,
                                                                  double* latency_us) {
    if (!valid_server(s) || !state) return fail(HCC_ERR_INVALID, "hcc_server_poll: invalid argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(HCC_ERR_INVALID, "hcc_server_poll: unknown request");
    *state = it->second.state;
    if (latency_us) {
        *latency_us = (it->second.state == kDone || it->second.state == kFailed)
                          ? std::chrono::duration<double, std::micro>(it->second.t_done - it->second.t_submit).count()
                          : -1.0;
    }
    return HCC_OK;
}

__attribute__((visibility("default"))) hcc_status hcc_server_cancel(hcc_server s, uint64_t id) {
    if (!valid_server(s)) return fail(HCC_ERR_INVALID, "hcc_server_cancel: invalid server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(HCC_ERR_INVALID, "hcc_server_cancel: unknown request");
    if (it->second.state != kQueued) return fail(HCC_ERR_INVALID, "hcc_server_cancel: request already admitted");
    it->second.state = kCancelled;
    return HCC_OK;
}

__attribute__((visibility("default"))) hcc_status hcc_server_drain(hcc_server s) {
    if (!valid_server(s)) return fail(HCC_ERR_INVALID, "hcc_server_drain: invalid server");
    while (true) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            bool busy = !s->inflight.empty() || s->running > 0;
            for (uint64_t id : s->pending)
                if (s->reqs[id].state == kQueued) busy = true;
            if (!busy) break;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    return HCC_OK;
}

__attribute__((visibility("default"))) hcc_status hcc_server_stats(hcc_server s, hcc_server_counters* out) {
    if (!valid_server(s) || !out) return fail(HCC_ERR_INVALID, "hcc_server_stats: invalid argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out->launches = s->launches;
    out->completed = s->completed;
    out->queued = 0;
    for (uint64_t id : s->pending)
        if (s->reqs[id].state == kQueued) out->queued += 1;
    out->running = s->running;
    out->used_bytes = s->used_bytes;
    return HCC_OK;
}

__attribute__((visibility("default"))) void hcc_server_destroy(hcc_server s) {
    if (!valid_server(s)) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (uint64_t id : s->pending) {
            Req& r = s->reqs[id];
            if (r.state == kQueued) r.state = kCancelled;
        }
        s->pending.clear();
        s->cv.notify_one();
    }
    s->worker.join();
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    for (auto& p : s->pinned_free) (void)hipHostFree(p.second);
    for (auto& sl : s->slots) {
        (void)hipGraphExecDestroy(sl.exec);
        s->alloc.put(sl.d_tables, nullptr);
        (void)hipHostFree(sl.pinned);
    }
    for (auto e : s->events_free) (void)hipEventDestroy(e);
    s->magic = 0;
    delete s;
}

}  // extern "C"
