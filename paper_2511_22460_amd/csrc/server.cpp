// Serving loop of libebr: single queries in, batches on the GPU, results out.
//
// Submitters append tickets to one FIFO queue. Each pipeline slot owns a HIP stream, a
// share of the caller's scratch arena and pinned staging, and a worker thread that takes
// the head of the queue as a batch (after an optional batching window), trims it to what
// the slot can hold, and runs the same top-K path as ebr_score_topk on it. With two or
// more slots a batch is formed and launched while the previous one is still on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace ebr {
namespace {

using Clock = std::chrono::steady_clock;

constexpr int kServerMaxBatch = 4096;
constexpr int kServerMaxPipeline = 4;
// Queued queries per batch of max_batch when the options leave the queue bound at 0.
constexpr int kDefaultQueueBatches = 16;
// Results per query the pinned staging is sized for (a batch with larger K holds fewer
// queries; one query of any allowed K always fits).
constexpr int kStagedK = 2048;

struct Ticket {
    uint64_t id = 0;
    const Index* ix = nullptr;  // the index the query runs on (the server's at submission)
    std::vector<float> user;
    std::vector<int32_t> keys;
    std::vector<float> mult;  // empty: all ones
    int32_t k = 0;
    uint64_t postings = 0;    // summed list length of its keys
    uint32_t* ids_out = nullptr;
    float* scores_out = nullptr;
    Clock::time_point t_submit;
    bool done = false;
    ebr_status status = EBR_OK;
    std::string err;
};

struct Slot {
    char* base = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    float* h_user = nullptr;    // pinned, max_batch x d
    uint32_t* h_ids = nullptr;  // pinned, out_cap
    float* h_scores = nullptr;  // pinned, out_cap
    ebr_graph* graph = nullptr; // the slot's captured-batch handle (graph option)
};

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace
}  // namespace ebr

using namespace ebr;

struct ebr_server {
    const Index* ix = nullptr;  // the current index: new queries run on it (guarded by mu)
    // per index: queries submitted to it and not yet completed (plus submissions in progress);
    // a swap waits until the previous index has none
    std::unordered_map<const Index*, int64_t> pending;
    int device = 0;
    ebr_server_opts opt{};
    int factor = 1;
    int64_t out_cap = 0;
    std::vector<Slot> slots;
    std::vector<std::thread> workers;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Ticket*> queue;
    std::unordered_map<uint64_t, Ticket*> tickets;
    uint64_t next_ticket = 1;
    bool stopping = false;

    uint64_t submitted = 0, completed = 0, failed = 0, batches = 0, batched = 0, rejected = 0;
    // fault injection for tests of the error path: the batch with this index (counted from 0
    // over the server's life) reports a device error instead of its results; -1: never
    int64_t fault_batch = -1;
    uint64_t batches_run = 0;
    std::vector<double> lat_ms;
    double busy_ms = 0.0;
    Clock::time_point t_stats;

    int kcount(const Index& x, int k) const {
        if (k == 0) return 0;
        return (int)std::min<int64_t>(x.n_ads, (int64_t)factor * k);
    }

    // Slot bytes a batch of these sizes needs on index x: user rows, both outputs, workspace.
    size_t need(const Index& x, const BatchSizes& z) const {
        return a256((size_t)z.B * x.dim * 4) + 2 * a256(4 * (size_t)std::max<int64_t>(1, z.n_out)) +
               topk_workspace_bytes(x, (int)opt.scan_dtype, z);
    }

    BatchSizes single(const Ticket& t) const {
        BatchSizes z;
        z.B = 1;
        z.nnz = (int64_t)t.keys.size();
        z.nu = (int)t.keys.size();
        z.bucket_n = t.postings;
        z.kcmax = kcount(*t.ix, t.k);
        z.n_out = t.k;
        return z;
    }

    void worker(int si);
    void run_batch(Slot& sl, std::vector<Ticket*>& take);
};

void ebr_server::worker(int si) {
    (void)hipSetDevice(device);
    Slot& sl = slots[si];
    const auto window = std::chrono::microseconds(std::max(0, opt.max_wait_us));
    for (;;) {
        std::vector<Ticket*> take;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stopping || !queue.empty(); });
            if (queue.empty()) {
                if (stopping) return;
                continue;
            }
            // batching window: wait for a full batch while the oldest query is young enough
            while (!stopping && !queue.empty() && (int)queue.size() < opt.max_batch) {
                const auto deadline = queue.front()->t_submit + window;
                if (Clock::now() >= deadline) break;
                cv_work.wait_until(lk, deadline);
            }
            if (queue.empty()) continue;
            // a batch runs on one index: the head's, up to the first query of a later one
            size_t n = std::min<size_t>(queue.size(), (size_t)opt.max_batch);
            for (size_t i = 1; i < n; ++i)
                if (queue[i]->ix != queue.front()->ix) { n = i; break; }
            take.assign(queue.begin(), queue.begin() + n);
            queue.erase(queue.begin(), queue.begin() + n);
        }
        // admission: first-in first-out while the batch fits the slot
        size_t keep = 0;
        try {
            // users per key of the batch so far; a batch of several query groups places the
            // postings of a key with u users min(u, limit) times at most (split buckets)
            std::unordered_map<int32_t, uint32_t> users;
            const Index& bx = *take[0]->ix;
            const int gq = score_group_queries(bx.dim);
            uint64_t distinct = 0, expanded = 0;
            int limit = 1;
            auto len = [&](int32_t k) { return (uint64_t)(bx.key_post_off[k + 1] - bx.key_post_off[k]); };
            BatchSizes z;
            for (; keep < take.size(); ++keep) {
                const Ticket& t = *take[keep];
                BatchSizes z2 = z;
                z2.B += 1;
                z2.nnz += (int64_t)t.keys.size();
                z2.n_out += t.k;
                z2.kcmax = std::max(z2.kcmax, kcount(bx, t.k));
                const int nqg = (z2.B + gq - 1) / gq;
                const int limit2 = split_groups(nqg) ? cold_user_limit(nqg) : 1;
                uint64_t distinct2 = distinct, expanded2 = expanded;
                if (limit2 != limit) {
                    expanded2 = 0;
                    for (const auto& kv : users) expanded2 += len(kv.first) * std::min<uint32_t>(kv.second, (uint32_t)limit2);
                }
                for (int32_t k : t.keys) {
                    const auto it = users.find(k);
                    const uint32_t c = it == users.end() ? 0u : it->second;
                    if (c == 0) {
                        z2.nu += 1;
                        distinct2 += len(k);
                    }
                    if (c < (uint32_t)limit2) expanded2 += len(k);
                }
                z2.bucket_n = limit2 > 1 ? expanded2 : distinct2;
                // the first query always fits (checked at submission)
                if (keep > 0 && (z2.n_out > out_cap || need(bx, z2) > sl.bytes)) break;
                for (int32_t k : t.keys) users[k] += 1;
                distinct = distinct2;
                expanded = expanded2;
                limit = limit2;
                z = z2;
            }
        } catch (const std::bad_alloc&) {
            keep = 1;
        }
        if (keep < take.size()) {
            std::lock_guard<std::mutex> lk(mu);
            queue.insert(queue.begin(), take.begin() + keep, take.end());
            take.resize(keep);
            cv_work.notify_all();
        }
        run_batch(sl, take);
    }
}

void ebr_server::run_batch(Slot& sl, std::vector<Ticket*>& take) {
    const auto t0 = Clock::now();
    const int B = (int)take.size();
    const Index& bx = *take[0]->ix;  // every query of a batch runs on the same index
    const int d = bx.dim;
    ebr_status st = EBR_OK;
    std::string err;
    try {
        std::vector<int64_t> offs(B + 1, 0);
        std::vector<int32_t> keys, kk(B);
        std::vector<float> mult;
        bool any_mult = false;
        for (const Ticket* t : take) any_mult |= !t->mult.empty();
        for (int i = 0; i < B; ++i) {
            const Ticket& t = *take[i];
            std::memcpy(sl.h_user + (size_t)i * d, t.user.data(), 4 * (size_t)d);
            keys.insert(keys.end(), t.keys.begin(), t.keys.end());
            if (any_mult) {
                if (t.mult.empty()) mult.insert(mult.end(), t.keys.size(), 1.0f);
                else mult.insert(mult.end(), t.mult.begin(), t.mult.end());
            }
            offs[i + 1] = (int64_t)keys.size();
            kk[i] = t.k;
        }
        int64_t n_out = 0;
        for (int i = 0; i < B; ++i) n_out += kk[i];
        char* p = sl.base;
        float* d_user = (float*)p;
        p += a256((size_t)B * d * 4);
        uint32_t* d_ids = (uint32_t*)p;
        p += a256(4 * (size_t)std::max<int64_t>(1, n_out));
        float* d_scores = (float*)p;
        p += a256(4 * (size_t)std::max<int64_t>(1, n_out));
        const size_t ws_bytes = sl.bytes - (size_t)(p - sl.base);
        hipError_t he = hipMemcpyAsync(d_user, sl.h_user, 4 * (size_t)B * d, hipMemcpyHostToDevice, sl.stream);
        if (he != hipSuccess) {
            set_error("hipMemcpyAsync (user rows) failed: %s", hipGetErrorString(he));
            st = EBR_EDEVICE;
        }
        if (!st) {
            ebr_batch bt{};
            bt.n_queries = B;
            bt.user_emb = d_user;
            bt.feat_offsets = offs.data();
            bt.feat_keys = keys.empty() ? nullptr : keys.data();
            bt.feat_mult = any_mult ? mult.data() : nullptr;
            bt.k = kk.data();
            // small batches may take the FP32 scan: its per-lane path for small query groups
            // is faster there, and a rescored query has the FP32 scan's result bits anyway
            const bool f32 = B <= opt.f32_below;
            bt.scan_dtype = f32 ? EBR_F32 : opt.scan_dtype;
            bt.rescore_factor = f32 ? 0 : factor;
            ebr_timings tm{};
            st = run_topk(bx, &bt, p, ws_bytes, d_ids, d_scores, sl.stream, &tm, sl.graph);
        }
        bool inject = false;
        {
            std::lock_guard<std::mutex> lk(mu);
            inject = fault_batch >= 0 && (int64_t)batches_run == fault_batch;
            ++batches_run;
        }
        if (!st && inject) {
            (void)hipStreamSynchronize(sl.stream);
            set_error("device step failed (fault injected by EBR_FAULT_BATCH for batch %lld)",
                      (long long)fault_batch);
            st = EBR_EDEVICE;
        }
        if (!st && n_out > 0) {
            he = hipMemcpyAsync(sl.h_ids, d_ids, 4 * (size_t)n_out, hipMemcpyDeviceToHost, sl.stream);
            if (he == hipSuccess)
                he = hipMemcpyAsync(sl.h_scores, d_scores, 4 * (size_t)n_out, hipMemcpyDeviceToHost, sl.stream);
            if (he == hipSuccess) he = hipStreamSynchronize(sl.stream);
            if (he != hipSuccess) {
                set_error("result copy failed: %s", hipGetErrorString(he));
                st = EBR_EDEVICE;
            }
        }
        if (!st) {
            int64_t pos = 0;
            for (Ticket* t : take) {
                if (t->k > 0) {
                    std::memcpy(t->ids_out, sl.h_ids + pos, 4 * (size_t)t->k);
                    std::memcpy(t->scores_out, sl.h_scores + pos, 4 * (size_t)t->k);
                }
                pos += t->k;
            }
        }
    } catch (const std::bad_alloc&) {
        set_error("host out of memory");
        st = EBR_ENOMEM;
    }
    if (st) err = last_error();
    const auto t1 = Clock::now();
    {
        std::lock_guard<std::mutex> lk(mu);
        for (Ticket* t : take) {
            t->done = true;
            --pending[t->ix];
            t->status = st;
            if (st) {
                t->err = err;
                ++failed;
            } else {
                ++completed;
                lat_ms.push_back(ms_between(t->t_submit, t1));
            }
        }
        ++batches;
        batched += (uint64_t)B;
        busy_ms += ms_between(t0, t1);
    }
    cv_done.notify_all();
}

extern "C" {

ebr_status ebr_server_create(const ebr_index* index, void* scratch, size_t scratch_bytes,
                             const ebr_server_opts* opts, ebr_server** out) {
    if (!index || !out || !opts) { set_error("NULL argument"); return EBR_EINVAL; }
    *out = nullptr;
    if (!scratch || ((uintptr_t)scratch & 255)) { set_error("scratch must be a 256-byte aligned device pointer"); return EBR_EINVAL; }
    ebr_server_opts o = *opts;
    if (o.max_batch == 0) o.max_batch = 256;
    if (o.pipeline == 0) o.pipeline = 2;
    if (o.max_wait_us < 0) o.max_wait_us = 0;
    if (o.f32_below < 0) o.f32_below = 0;
    if (o.max_queue == 0) o.max_queue = kDefaultQueueBatches * o.max_batch;
    if (o.max_queue < 1) { set_error("max_queue must be >= 1 (0: the default)"); return EBR_EINVAL; }
    if (o.max_batch < 1 || o.max_batch > kServerMaxBatch) { set_error("max_batch must be in [1, %d]", kServerMaxBatch); return EBR_EINVAL; }
    if (o.pipeline < 1 || o.pipeline > kServerMaxPipeline) { set_error("pipeline must be in [1, %d]", kServerMaxPipeline); return EBR_EINVAL; }
    if (o.scan_dtype != EBR_F32 && o.scan_dtype != EBR_BF16 && o.scan_dtype != EBR_FP8E4M3) { set_error("unknown scan dtype"); return EBR_EINVAL; }
    const Index& ix = *index;
    if ((o.scan_dtype == EBR_BF16 && !ix.emb_bf16) || (o.scan_dtype == EBR_FP8E4M3 && !ix.emb_fp8)) {
        set_error("the index holds no copy of the requested scan dtype");
        return EBR_EUNSUPPORTED;
    }
    ebr_server* S = nullptr;
    try {
        S = new ebr_server();
        S->ix = &ix;
        S->opt = o;
        S->factor = o.scan_dtype == EBR_F32 ? 1 : (o.rescore_factor > 0 ? o.rescore_factor : 4);
        if (S->factor > kMaxK) { delete S; set_error("rescore_factor too large"); return EBR_EINVAL; }
        S->out_cap = (int64_t)o.max_batch * std::min<int64_t>(ix.n_ads, kStagedK) + std::min<int64_t>(ix.n_ads, kMaxK);
        if (hipGetDevice(&S->device) != hipSuccess) { delete S; set_error("hipGetDevice failed"); return EBR_EDEVICE; }
        const size_t per = (scratch_bytes / (size_t)o.pipeline) & ~(size_t)255;
        BatchSizes z1;
        z1.B = 1;
        z1.kcmax = 1;
        z1.n_out = 1;
        if (S->need(ix, z1) > per) {
            set_error("scratch of %zu bytes per slot cannot hold a one-query batch (%zu bytes)", per, S->need(ix, z1));
            delete S;
            return EBR_ENOMEM;
        }
        S->slots.resize(o.pipeline);
        auto fail = [&](const char* what, hipError_t e) {
            set_error("%s failed: %s", what, hipGetErrorString(e));
            for (Slot& sl : S->slots) {
                if (sl.graph) ebr_graph_destroy(sl.graph);
                if (sl.stream) (void)hipStreamDestroy(sl.stream);
                if (sl.h_user) (void)hipHostFree(sl.h_user);
                if (sl.h_ids) (void)hipHostFree(sl.h_ids);
                if (sl.h_scores) (void)hipHostFree(sl.h_scores);
            }
            delete S;
            return EBR_EDEVICE;
        };
        for (int i = 0; i < o.pipeline; ++i) {
            Slot& sl = S->slots[i];
            sl.base = (char*)scratch + (size_t)i * per;
            sl.bytes = per;
            hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
            if (e != hipSuccess) return fail("hipStreamCreateWithFlags", e);
            e = hipHostMalloc((void**)&sl.h_user, 4 * (size_t)o.max_batch * ix.dim, hipHostMallocDefault);
            if (e != hipSuccess) return fail("hipHostMalloc", e);
            e = hipHostMalloc((void**)&sl.h_ids, 4 * (size_t)S->out_cap, hipHostMallocDefault);
            if (e != hipSuccess) return fail("hipHostMalloc", e);
            e = hipHostMalloc((void**)&sl.h_scores, 4 * (size_t)S->out_cap, hipHostMallocDefault);
            if (e != hipSuccess) return fail("hipHostMalloc", e);
            if (o.graph && ebr_graph_create(&sl.graph) != EBR_OK) return fail("ebr_graph_create", hipErrorUnknown);
        }
        S->t_stats = Clock::now();
        if (const char* f = std::getenv("EBR_FAULT_BATCH")) {
            char* end = nullptr;
            const long long v = std::strtoll(f, &end, 10);
            if (end != f && *end == '\0' && v >= 0) S->fault_batch = v;
        }
        for (int i = 0; i < o.pipeline; ++i) S->workers.emplace_back([S, i] { S->worker(i); });
    } catch (const std::exception&) {
        set_error("host out of resources");
        if (S) {
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->stopping = true;
            }
            S->cv_work.notify_all();
            for (auto& w : S->workers) w.join();
            for (Slot& sl : S->slots) {
                if (sl.graph) ebr_graph_destroy(sl.graph);
                if (sl.stream) (void)hipStreamDestroy(sl.stream);
                if (sl.h_user) (void)hipHostFree(sl.h_user);
                if (sl.h_ids) (void)hipHostFree(sl.h_ids);
                if (sl.h_scores) (void)hipHostFree(sl.h_scores);
            }
            delete S;
        }
        return EBR_ENOMEM;
    }
    *out = S;
    return EBR_OK;
}

static ebr_status submit_on(ebr_server* S, const Index& ix, const ebr_query* q, uint32_t* ids_out,
                            float* scores_out, uint64_t* ticket);

ebr_status ebr_submit(ebr_server* S, const ebr_query* q, uint32_t* ids_out, float* scores_out,
                      uint64_t* ticket) {
    if (!S || !q || !ticket) { set_error("NULL argument"); return EBR_EINVAL; }
    // the index of this submission stays alive until it is released below or the query has
    // completed (a swap waits for both)
    const Index* cur = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        cur = S->ix;
        ++S->pending[cur];
    }
    auto release = [&](ebr_status s) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            --S->pending[cur];
        }
        S->cv_done.notify_all();
        return s;
    };
    const ebr_status r = submit_on(S, *cur, q, ids_out, scores_out, ticket);
    return r == EBR_OK ? r : release(r);
}

static ebr_status submit_on(ebr_server* S, const Index& ix, const ebr_query* q, uint32_t* ids_out,
                            float* scores_out, uint64_t* ticket) {
    if (!q->user_emb) { set_error("user_emb is NULL"); return EBR_EINVAL; }
    if (q->n_feats < 0 || (q->n_feats > 0 && !q->feat_keys)) { set_error("bad feature list"); return EBR_EINVAL; }
    const int64_t kcap = std::min<int64_t>(ix.n_ads, kMaxK / S->factor);
    if (q->k < 0 || q->k > kcap) { set_error("K = %d outside [0, %lld]", q->k, (long long)kcap); return EBR_EINVAL; }
    if (q->k > 0 && (!ids_out || !scores_out)) { set_error("NULL output"); return EBR_EINVAL; }
    try {
        Ticket* t = new Ticket();
        t->user.assign(q->user_emb, q->user_emb + ix.dim);
        t->keys.assign(q->feat_keys, q->feat_keys + q->n_feats);
        if (q->feat_mult) t->mult.assign(q->feat_mult, q->feat_mult + q->n_feats);
        t->k = q->k;
        t->ix = &ix;
        t->ids_out = ids_out;
        t->scores_out = scores_out;
        auto reject = [&](ebr_status s) { delete t; return s; };
        for (float v : t->user)
            if (!std::isfinite(v)) { set_error("non-finite user embedding"); return reject(EBR_EINVAL); }
        for (float v : t->mult)
            if (!std::isfinite(v)) { set_error("non-finite multiplier"); return reject(EBR_EINVAL); }
        std::vector<int32_t> sk(t->keys);
        std::sort(sk.begin(), sk.end());
        if (!sk.empty() && (sk.front() < 0 || sk.back() >= ix.n_keys)) { set_error("key out of range [0, %lld)", (long long)ix.n_keys); return reject(EBR_EINVAL); }
        if (std::adjacent_find(sk.begin(), sk.end()) != sk.end()) { set_error("query repeats a key"); return reject(EBR_EINVAL); }
        for (int32_t k : sk) t->postings += (uint64_t)(ix.key_post_off[k + 1] - ix.key_post_off[k]);
        const size_t need = S->need(ix, S->single(*t));
        if (need > S->slots[0].bytes) {
            set_error("query needs %zu bytes of scratch, a slot holds %zu", need, S->slots[0].bytes);
            return reject(EBR_ENOMEM);
        }
        t->t_submit = Clock::now();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->stopping) { set_error("server is shutting down"); return reject(EBR_ESHUTDOWN); }
            if ((int64_t)S->queue.size() >= (int64_t)S->opt.max_queue) {
                ++S->rejected;
                set_error("queue full (%d queries waiting); poll and submit again", S->opt.max_queue);
                return reject(EBR_EAGAIN);
            }
            t->id = S->next_ticket++;
            S->tickets[t->id] = t;
            S->queue.push_back(t);
            ++S->submitted;
            *ticket = t->id;
        }
        S->cv_work.notify_all();
        return EBR_OK;
    } catch (const std::bad_alloc&) {
        set_error("host out of memory");
        return EBR_ENOMEM;
    }
}

ebr_status ebr_server_swap_index(ebr_server* S, const ebr_index* next) {
    if (!S || !next) { set_error("NULL argument"); return EBR_EINVAL; }
    const Index* old = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        old = S->ix;
    }
    if (next->dim != old->dim || next->n_ads != old->n_ads) {
        set_error("the new index must have the same ads and width (%lld x %d), not %lld x %d",
                  (long long)old->n_ads, old->dim, (long long)next->n_ads, next->dim);
        return EBR_EINVAL;
    }
    if ((S->opt.scan_dtype == EBR_BF16 && !next->emb_bf16) || (S->opt.scan_dtype == EBR_FP8E4M3 && !next->emb_fp8)) {
        set_error("the new index lacks the server's scan copy");
        return EBR_EUNSUPPORTED;
    }
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->ix != old) { set_error("another swap is in progress"); return EBR_EAGAIN; }
    S->ix = next;
    S->cv_done.wait(lk, [&] { return S->pending[old] == 0; });
    if (next != old) S->pending.erase(old);
    return EBR_OK;
}

ebr_status ebr_poll(ebr_server* S, uint64_t ticket, int32_t timeout_us) {
    if (!S) { set_error("NULL argument"); return EBR_EINVAL; }
    std::unique_lock<std::mutex> lk(S->mu);
    auto ready = [&] {
        auto it = S->tickets.find(ticket);
        return it == S->tickets.end() || it->second->done;
    };
    if (timeout_us < 0) S->cv_done.wait(lk, ready);
    else if (timeout_us > 0) S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) { set_error("unknown ticket %llu", (unsigned long long)ticket); return EBR_ENOTFOUND; }
    Ticket* t = it->second;
    if (!t->done) return EBR_EAGAIN;
    const ebr_status st = t->status;
    const std::string err = t->err;
    S->tickets.erase(it);
    lk.unlock();
    delete t;
    if (st) set_error("%s", err.c_str());
    return st;
}

ebr_status ebr_server_stats(ebr_server* S, ebr_server_info* out) {
    if (!S || !out) { set_error("NULL argument"); return EBR_EINVAL; }
    std::vector<double> lat;
    ebr_server_info r{};
    {
        std::lock_guard<std::mutex> lk(S->mu);
        lat = S->lat_ms;
        r.submitted = S->submitted;
        r.completed = S->completed;
        r.failed = S->failed;
        r.queued = S->queue.size();
        r.rejected = S->rejected;
        r.batches = S->batches;
        r.mean_batch = S->batches ? (double)S->batched / (double)S->batches : 0.0;
        r.busy_ms = S->busy_ms;
        r.elapsed_ms = ms_between(S->t_stats, Clock::now());
    }
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        const size_t n = lat.size();
        // nearest-rank percentiles
        auto pct = [&](double p) { return lat[(size_t)std::max(0.0, std::ceil(p * (double)n) - 1.0)]; };
        r.p50_ms = pct(0.50);
        r.p99_ms = pct(0.99);
        r.max_ms = lat.back();
        double sum = 0.0;
        for (double v : lat) sum += v;
        r.mean_ms = sum / (double)n;
    }
    r.qps = r.elapsed_ms > 0.0 ? (double)r.completed / (r.elapsed_ms * 1e-3) : 0.0;
    *out = r;
    return EBR_OK;
}

ebr_status ebr_server_reset_stats(ebr_server* S) {
    if (!S) { set_error("NULL argument"); return EBR_EINVAL; }
    std::lock_guard<std::mutex> lk(S->mu);
    S->completed = S->failed = S->batches = S->batched = S->rejected = 0;
    S->submitted = S->queue.size();
    S->lat_ms.clear();
    S->busy_ms = 0.0;
    S->t_stats = Clock::now();
    return EBR_OK;
}

ebr_status ebr_server_destroy(ebr_server* S) {
    if (!S) { set_error("NULL argument"); return EBR_EINVAL; }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    for (auto& w : S->workers) w.join();
    ebr_status st = EBR_OK;
    for (Slot& sl : S->slots) {
        if (sl.graph) ebr_graph_destroy(sl.graph);
        if (sl.stream && hipStreamDestroy(sl.stream) != hipSuccess) st = EBR_EDEVICE;
        if (sl.h_user) (void)hipHostFree(sl.h_user);
        if (sl.h_ids) (void)hipHostFree(sl.h_ids);
        if (sl.h_scores) (void)hipHostFree(sl.h_scores);
    }
    for (auto& kv : S->tickets) delete kv.second;
    delete S;
    if (st) set_error("hipStreamDestroy failed");
    return st;
}

}  // extern "C"
