// Host runtime and C ABI of libebr: input validation, index build (encode + upload into the
// caller's arena), batch planning, and the launch sequence of one top-K batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "build.h"
#include "kernels.h"

namespace ebr {

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}
const char* last_error() { return g_err.c_str(); }

#define HIP_TRY(expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (hipError_t)(expr);                                        \
        if (e_ != hipSuccess) {                                                    \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));              \
            return EBR_EDEVICE;                                                    \
        }                                                                          \
    } while (0)

#define LAUNCH(expr)                                                                       \
    do {                                                                                   \
        int rc_ = (expr);                                                                  \
        if (rc_) {                                                                         \
            set_error("%s failed: %s", #expr, hipGetErrorString((hipError_t)rc_));         \
            return EBR_EDEVICE;                                                            \
        }                                                                                  \
    } while (0)

// ------------------------------------------------------------------ phase timing

static std::atomic<int> g_timing{0};
static thread_local ebr_timings g_last_timings{};

// HIP events recorded on the call's stream at phase boundaries (only while timing is on).
struct PhaseClock {
    bool on = false;
    hipStream_t st = nullptr;
    std::vector<hipEvent_t> ev;
    PhaseClock(hipStream_t s, bool enable) : on(enable), st(s) {}
    ~PhaseClock() { for (hipEvent_t e : ev) (void)hipEventDestroy(e); }
    int mark() {  // returns the event index, or -1 when timing is off
        if (!on) return -1;
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { on = false; return -1; }
        ev.push_back(e);
        if (hipEventRecord(e, st) != hipSuccess) { on = false; return -1; }
        return (int)ev.size() - 1;
    }
    double ms(int a, int b) const {
        if (!on || a < 0 || b < 0) return 0.0;
        float t = 0.0f;
        if (hipEventElapsedTime(&t, ev[a], ev[b]) != hipSuccess) return 0.0;
        return (double)t;
    }
};

// ------------------------------------------------------------------ host threading

// Host threads for the planner and the index encoder: the machine's, at most 16 (the CPU
// share of one GPU on the hosts served).
static int host_threads() {
    unsigned n = std::thread::hardware_concurrency();
    if (n == 0) n = 4;
    return (int)std::min(n, 16u);
}

// Persistent workers for the planner's parallel loops (a thread per slice would cost tens of
// microseconds to start, several times per batch). One loop runs on the pool at a time; a
// loop started while the pool is busy (another batch being planned on another thread) runs
// its slices with threads of its own.
class HostPool {
  public:
    explicit HostPool(int n) {
        for (int i = 0; i < n; ++i) workers_.emplace_back([this] { work(); });
    }
    ~HostPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : workers_) t.join();
    }
    int size() const { return (int)workers_.size(); }
    // fn(t) for t in [0, n): the caller runs slice 0, the workers the rest; false if busy
    bool run(int n, const std::function<void(int)>& fn) {
        std::unique_lock<std::mutex> busy(run_mu_, std::try_to_lock);
        if (!busy.owns_lock()) return false;
        {
            std::lock_guard<std::mutex> lk(mu_);
            fn_ = &fn;
            n_ = n;
            next_ = 1;
            left_ = n - 1;
            ++gen_;
        }
        cv_.notify_all();
        fn(0);
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [this] { return left_ == 0; });
        fn_ = nullptr;
        return true;
    }

  private:
    void work() {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_.wait(lk, [&] { return stop_ || (gen_ != seen && next_ < n_); });
            if (stop_) return;
            seen = gen_;
            while (next_ < n_) {
                const int t = next_++;
                const std::function<void(int)>* f = fn_;
                lk.unlock();
                (*f)(t);
                lk.lock();
                if (--left_ == 0) done_.notify_all();
            }
        }
    }
    std::vector<std::thread> workers_;
    std::mutex mu_, run_mu_;
    std::condition_variable cv_, done_;
    const std::function<void(int)>* fn_ = nullptr;
    int n_ = 0, next_ = 0, left_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

static HostPool& host_pool() {
    static HostPool pool(host_threads() - 1);
    return pool;
}

// Calls fn(begin, end) on nt contiguous slices of [0, n).
static void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& fn,
                         int64_t min_per_thread = 4096) {
    int nt = host_threads();
    if (n < min_per_thread * 2) nt = 1;
    if (nt <= 1) { fn(0, n); return; }
    const int64_t per = (n + nt - 1) / nt;
    const int ns = (int)((n + per - 1) / per);
    auto slice = [&](int t) {
        const int64_t b = t * per, e = std::min(n, b + per);
        if (b < e) fn(b, e);
    };
    if (host_pool().run(ns, slice)) return;
    std::vector<std::thread> th;
    for (int t = 1; t < ns; ++t) th.emplace_back(slice, t);
    slice(0);
    for (auto& x : th) x.join();
}

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ------------------------------------------------------------------ index build

struct Measured {
    std::vector<uint32_t> key_chunk_off;  // V + 1
    std::vector<uint64_t> key_word_off;   // V + 1
    ArenaPlan plan;
};

static bool dim_ok(int32_t d) { return d >= 16 && d <= 128 && d % 16 == 0 && score_dim_supported(d); }

static ebr_status validate_desc(const ebr_build_desc* d) {
    if (!d) { set_error("desc is NULL"); return EBR_EINVAL; }
    if (d->n_ads < 1 || d->n_ads > 0xffffffffLL) { set_error("n_ads must be in [1, 2^32)"); return EBR_EINVAL; }
    if (!dim_ok(d->dim)) { set_error("dim %d unsupported: need a multiple of 16 in [16, 128]", d->dim); return EBR_EINVAL; }
    if (!d->ad_emb) { set_error("ad_emb is NULL"); return EBR_EINVAL; }
    if (d->n_keys < 0) { set_error("n_keys < 0"); return EBR_EINVAL; }
    if (d->n_keys > 0 && !d->key_offsets) { set_error("key_offsets is NULL"); return EBR_EINVAL; }
    if (d->dtypes & ~7u) { set_error("unknown dtype bits in %u", d->dtypes); return EBR_EINVAL; }
    const int64_t V = d->n_keys;
    if (V > 0) {
        if (d->key_offsets[0] != 0) { set_error("key_offsets[0] != 0"); return EBR_EINVAL; }
        for (int64_t k = 0; k < V; ++k)
            if (d->key_offsets[k + 1] < d->key_offsets[k]) { set_error("key_offsets decrease at key %lld", (long long)k); return EBR_EINVAL; }
        const int64_t total = d->key_offsets[V];
        if (total > 0xffffffffLL - 64) { set_error("more than 2^32 postings"); return EBR_EINVAL; }
        if (total > 0 && !d->post_ids) { set_error("post_ids is NULL"); return EBR_EINVAL; }
    }
    std::atomic<int64_t> bad_key{-1}, bad_w{-1}, bad_row{-1};
    if (V > 0) {
        parallel_for(V, [&](int64_t b, int64_t e) {
            for (int64_t k = b; k < e; ++k) {
                const int64_t s = d->key_offsets[k], t = d->key_offsets[k + 1];
                for (int64_t i = s; i < t; ++i) {
                    if (d->post_ids[i] >= (uint64_t)d->n_ads || (i > s && d->post_ids[i] <= d->post_ids[i - 1])) {
                        bad_key = k;
                        break;
                    }
                    if (d->post_w && !std::isfinite(d->post_w[i])) { bad_w = k; break; }
                }
            }
        }, 256);
    }
    if (bad_key >= 0) { set_error("postings of key %lld are not strictly increasing ids < n_ads", (long long)bad_key.load()); return EBR_EINVAL; }
    if (bad_w >= 0) { set_error("non-finite weight in key %lld", (long long)bad_w.load()); return EBR_EINVAL; }
    parallel_for(d->n_ads, [&](int64_t b, int64_t e) {
        for (int64_t a = b; a < e; ++a)
            for (int32_t i = 0; i < d->dim; ++i)
                if (!std::isfinite(d->ad_emb[a * d->dim + i])) { bad_row = a; return; }
    });
    if (bad_row >= 0) { set_error("non-finite embedding in ad %lld", (long long)bad_row.load()); return EBR_EINVAL; }
    return EBR_OK;
}

static ebr_status measure(const ebr_build_desc* d, Measured* m) {
    const int64_t V = d->n_keys;
    std::vector<int64_t> ch(V), wd(V);
    if (V > 0) {
        parallel_for(V, [&](int64_t b, int64_t e) {
            for (int64_t k = b; k < e; ++k) {
                const int64_t s = d->key_offsets[k], t = d->key_offsets[k + 1];
                codec_measure(d->post_ids + s, t - s, &ch[k], &wd[k]);
            }
        }, 256);
    }
    m->key_chunk_off.assign(V + 1, 0);
    m->key_word_off.assign(V + 1, 0);
    uint64_t c = 0, w = 0;
    for (int64_t k = 0; k < V; ++k) {
        m->key_chunk_off[k] = (uint32_t)c;
        m->key_word_off[k] = w;
        c += (uint64_t)ch[k];
        w += (uint64_t)wd[k];
        if (c > 0xffffffffull || w > 0xfffffff0ull) { set_error("index too large for 32-bit chunk/word offsets"); return EBR_EINVAL; }
    }
    m->key_chunk_off[V] = (uint32_t)c;
    m->key_word_off[V] = w;
    const int64_t n_post = V > 0 ? d->key_offsets[V] : 0;
    m->plan = arena_plan(d->n_ads, d->dim, d->dtypes, n_post, (int64_t)c, (int64_t)w, d->post_w != nullptr);
    return EBR_OK;
}

ArenaPlan arena_plan(int64_t n_ads, int32_t dim, uint32_t dtypes, int64_t n_post, int64_t n_chunks,
                     int64_t n_words, bool weights) {
    ArenaPlan p;
    const int64_t n_blk = (n_ads + kTileAds - 1) / kTileAds;
    p.n_chunks = n_chunks;
    p.n_words = n_words;
    p.bytes_emb_f32 = (size_t)n_blk * kTileAds * dim * 4;
    p.bytes_chunks = std::max<size_t>(16, (size_t)n_chunks * 16);
    p.bytes_words = (size_t)(n_words + 2) * 4;
    // an index without weights (the paper's binary L) stores ids only
    p.bytes_weights = weights ? std::max<size_t>(4, (size_t)n_post * 4) : 0;
    size_t off = 0;
    p.off_emb_f32 = off; off = align256(off + p.bytes_emb_f32);
    if (dtypes & (1u << EBR_BF16)) {
        p.bytes_emb_bf16 = (size_t)n_blk * kTileAds * dim * 2;
        p.off_emb_bf16 = off; off = align256(off + p.bytes_emb_bf16);
    }
    if (dtypes & (1u << EBR_FP8E4M3)) {
        p.bytes_emb_fp8 = (size_t)n_blk * kTileAds * dim;
        p.off_emb_fp8 = off; off = align256(off + p.bytes_emb_fp8);
        p.bytes_fp8_scale = (size_t)n_blk * kTileAds * 4;
        p.off_fp8_scale = off; off = align256(off + p.bytes_fp8_scale);
    }
    p.off_chunks = off; off = align256(off + p.bytes_chunks);
    p.off_words = off; off = align256(off + p.bytes_words);
    p.off_weights = off;
    if (p.bytes_weights) off = align256(off + p.bytes_weights);
    p.total = off;
    return p;
}

// FP32 copy: the rows, row-major, padded with zero rows to a multiple of 32 (k_score stages
// a tile's 32 rows into the matrix-core operand order in LDS; a rescored ad's row is
// contiguous).
static void swizzle_f32(const float* E, int64_t n_ads, int32_t d, float* out) {
    const int64_t n_blk = (n_ads + kTileAds - 1) / kTileAds;
    parallel_for(n_blk, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            float* dst = out + b * (int64_t)kTileAds * d;
            for (int l = 0; l < kTileAds; ++l) {
                const int64_t row = b * kTileAds + l;
                if (row < n_ads) std::memcpy(dst + (int64_t)l * d, E + row * d, sizeof(float) * (size_t)d);
                else std::memset(dst + (int64_t)l * d, 0, sizeof(float) * (size_t)d);
            }
        }
    }, 64);
}

// The index object over a filled arena (host build and device build alike).
static ebr_index* finish_index(int64_t n_ads, int32_t dim, uint32_t dtypes, int64_t V, int64_t n_post, bool has_w,
                               const ArenaPlan& p, char* base, std::vector<uint32_t> key_chunk_off,
                               const int64_t* key_offsets, std::vector<float> maxw, const double* q_err2,
                               const double* q_norm2, double e_norm2, double enc_ms, double up_ms) {
    ebr_index* ix = new ebr_index();
    ix->n_ads = n_ads;
    ix->n_keys = V;
    ix->n_postings = n_post;
    ix->n_chunks = p.n_chunks;
    ix->dim = dim;
    ix->n_tiles = (n_ads + kTileAds - 1) / kTileAds;
    ix->dtypes = 1u | dtypes;
    ix->emb_f32 = base + p.off_emb_f32;
    if ((dtypes & (1u << EBR_BF16))) ix->emb_bf16 = base + p.off_emb_bf16;
    if ((dtypes & (1u << EBR_FP8E4M3))) {
        ix->emb_fp8 = base + p.off_emb_fp8;
        ix->fp8_scale = (const float*)(base + p.off_fp8_scale);
    }
    for (int c = 0; c < 2; ++c) { ix->q_err2[c] = q_err2[c]; ix->q_norm2[c] = q_norm2[c]; }
    ix->e_norm2 = e_norm2;
    ix->chunks = (const ChunkHdr*)(base + p.off_chunks);
    ix->words = (const uint32_t*)(base + p.off_words);
    ix->weights = has_w ? (const float*)(base + p.off_weights) : nullptr;  // null: W = 1
    ix->key_chunk_off = std::move(key_chunk_off);
    ix->key_post_off.assign(key_offsets ? key_offsets : nullptr, key_offsets ? key_offsets + V + 1 : nullptr);
    if (ix->key_post_off.empty()) ix->key_post_off.assign(1, 0);
    ix->key_maxw = std::move(maxw);
    // per-key weight scale: |w| * 2^Sw < 2^30 with max |w| * 2^Sw >= 2^29
    ix->key_wshift.assign((size_t)V, 0);
    for (int64_t k = 0; k < V; ++k) {
        if (ix->key_maxw[k] > 0.0f) {
            int e;
            std::frexp((double)ix->key_maxw[k], &e);  // max|w| < 2^e
            ix->key_wshift[k] = (int8_t)std::max(-120, std::min(120, 30 - e));
        }
    }
    if (hipGetDevice(&ix->device) != hipSuccess) ix->device = 0;
    ebr_index_info& s = ix->stats;
    s.n_ads = ix->n_ads;
    s.n_keys = V;
    s.n_postings = n_post;
    s.n_chunks = p.n_chunks;
    s.n_tiles = ix->n_tiles;
    s.dim = ix->dim;
    s.tile_ads = kTileAds;
    s.arena_bytes = p.total;
    s.bytes_emb_f32 = p.bytes_emb_f32;
    s.bytes_emb_bf16 = p.bytes_emb_bf16;
    s.bytes_emb_fp8 = p.bytes_emb_fp8 + p.bytes_fp8_scale;
    s.max_err_bf16 = q_err2[0];
    s.max_err_fp8 = q_err2[1];
    s.bytes_chunk_headers = (uint64_t)p.n_chunks * 16;
    s.bytes_packed_ids = (uint64_t)p.n_words * 4;
    s.bytes_weights = has_w ? (uint64_t)n_post * 4 : 0;
    s.bits_per_id = n_post ? (double)(s.bytes_chunk_headers + s.bytes_packed_ids) * 8.0 / (double)n_post : 0.0;
    s.bytes_per_posting = n_post ? (double)(s.bytes_chunk_headers + s.bytes_packed_ids + s.bytes_weights) / (double)n_post : 0.0;
    s.encode_ms = enc_ms;
    s.upload_ms = up_ms;
    return ix;
}

// ------------------------------------------------------------------ device build (refresh)


// Scratch sections of a device build of n_keys lists holding n_post postings.
struct BuildScratch {
    size_t o_kc = 0, o_kco = 0, o_maxw = 0, o_ck = 0, o_cw = 0, o_wo = 0, o_ci = 0, o_flags = 0, o_stats = 0,
           o_tmp = 0, total = 0;
};

static BuildScratch build_scratch(int64_t V, int64_t n_post) {
    BuildScratch b;
    const int64_t chunks = n_post / kChunk + V + 1;  // sum over lists of ceil(L / 64)
    size_t off = 0;
    auto put = [&](size_t bytes) { size_t o = off; off = align256(off + std::max<size_t>(bytes, 16)); return o; };
    b.o_kc = put(4 * (size_t)(V + 1));
    b.o_kco = put(4 * (size_t)(V + 1));
    b.o_maxw = put(4 * (size_t)std::max<int64_t>(1, V));
    b.o_ck = put(4 * (size_t)chunks);
    b.o_cw = put(4 * (size_t)(chunks + 1));
    b.o_wo = put(4 * (size_t)(chunks + 1));
    b.o_ci = put(4 * (size_t)chunks);
    b.o_flags = put(16);
    b.o_stats = put(64);
    b.o_tmp = put(4 * (size_t)scan_tmp_words(std::max<int64_t>(V, chunks) + 1));
    b.total = off;
    return b;
}

// Validate the host-visible sizes and the list offsets (copied to the host), then find every
// list's chunks and every chunk's shape on the device. Leaves the sizes in *n_chunks, *n_words.
static ebr_status device_shapes(const ebr_build_desc* d, char* scr, size_t scr_bytes, hipStream_t st, BuildArgs* a,
                         std::vector<int64_t>* key_off, int64_t* n_chunks, int64_t* n_words) {
    if (!d) { set_error("desc is NULL"); return EBR_EINVAL; }
    if (d->n_ads < 1 || d->n_ads > 0xffffffffLL) { set_error("n_ads must be in [1, 2^32)"); return EBR_EINVAL; }
    if (!dim_ok(d->dim)) { set_error("dim %d unsupported: need a multiple of 16 in [16, 128]", d->dim); return EBR_EINVAL; }
    if (!d->ad_emb) { set_error("ad_emb is NULL"); return EBR_EINVAL; }
    if (d->n_keys < 0) { set_error("n_keys < 0"); return EBR_EINVAL; }
    if (d->n_keys > 0 && !d->key_offsets) { set_error("key_offsets is NULL"); return EBR_EINVAL; }
    if (d->dtypes & ~7u) { set_error("unknown dtype bits in %u", d->dtypes); return EBR_EINVAL; }
    const int64_t V = d->n_keys;
    key_off->assign((size_t)V + 1, 0);
    if (V > 0) {
        HIP_TRY(hipMemcpyAsync(key_off->data(), d->key_offsets, 8 * (size_t)(V + 1), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if ((*key_off)[0] != 0) { set_error("key_offsets[0] != 0"); return EBR_EINVAL; }
        for (int64_t k = 0; k < V; ++k)
            if ((*key_off)[k + 1] < (*key_off)[k]) { set_error("key_offsets decrease at key %lld", (long long)k); return EBR_EINVAL; }
        if ((*key_off)[V] > 0xffffffffLL - 64) { set_error("more than 2^32 postings"); return EBR_EINVAL; }
        if ((*key_off)[V] > 0 && !d->post_ids) { set_error("post_ids is NULL"); return EBR_EINVAL; }
    }
    const int64_t n_post = (*key_off)[V];
    const BuildScratch bs = build_scratch(V, n_post);
    if (!scr || scr_bytes < bs.total) { set_error("scratch too small: need %zu bytes, got %zu", bs.total, scr_bytes); return EBR_ENOMEM; }
    if ((uintptr_t)scr & 255) { set_error("scratch must be 256-byte aligned"); return EBR_EINVAL; }
    *a = BuildArgs{};
    a->n_ads = d->n_ads;
    a->dim = d->dim;
    a->n_keys = V;
    a->key_offsets = d->key_offsets;
    a->post_ids = d->post_ids;
    a->post_w = d->post_w;
    a->emb = d->ad_emb;
    a->key_chunks = (uint32_t*)(scr + bs.o_kc);
    a->key_chunk_off = (uint32_t*)(scr + bs.o_kco);
    a->key_maxw = (float*)(scr + bs.o_maxw);
    a->chunk_key = (uint32_t*)(scr + bs.o_ck);
    a->chunk_words = (uint32_t*)(scr + bs.o_cw);
    a->word_off = (uint32_t*)(scr + bs.o_wo);
    a->chunk_info = (uint32_t*)(scr + bs.o_ci);
    a->flags = (unsigned long long*)(scr + bs.o_flags);
    a->stats = (unsigned long long*)(scr + bs.o_stats);
    uint32_t* tmp = (uint32_t*)(scr + bs.o_tmp);
    LAUNCH(launch_fill_u32((uint32_t*)a->flags, 0xffffffffu, 4, st));
    LAUNCH(launch_fill_u32((uint32_t*)a->stats, 0u, 16, st));
    LAUNCH(launch_build_lists(*a, st));
    LAUNCH(launch_excl_scan_u32(a->key_chunks, a->key_chunk_off, V, tmp, st));
    unsigned long long bad = 0;
    uint32_t nc = 0;
    HIP_TRY(hipMemcpyAsync(&bad, a->flags, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&nc, a->key_chunk_off + V, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (bad != ~0ull) {
        set_error("postings of key %llu are not strictly increasing ids < n_ads with finite weights", bad);
        return EBR_EINVAL;
    }
    a->n_chunks = nc;
    LAUNCH(launch_build_chunks(*a, st));
    LAUNCH(launch_excl_scan_u32(a->chunk_words, a->word_off, nc, tmp, st));
    uint32_t nw = 0;
    HIP_TRY(hipMemcpyAsync(&nw, a->word_off + nc, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (nw > 0xfffffff0u) { set_error("index too large for 32-bit word offsets"); return EBR_EINVAL; }
    *n_chunks = nc;
    *n_words = nw;
    return EBR_OK;
}

}  // namespace ebr

using namespace ebr;

extern "C" {

const char* ebr_last_error(void) { return ebr::last_error(); }
const char* ebr_version(void) { return "libebr 0.1 (gfx950)"; }

ebr_status ebr_set_timing(int enable) {
    g_timing.store(enable ? 1 : 0);
    return EBR_OK;
}

ebr_status ebr_get_timings(ebr_timings* out) {
    if (!out) { set_error("out is NULL"); return EBR_EINVAL; }
    *out = g_last_timings;
    return EBR_OK;
}

ebr_status ebr_index_size(const ebr_build_desc* desc, size_t* arena_bytes) {
    try {
        if (!arena_bytes) { set_error("arena_bytes is NULL"); return EBR_EINVAL; }
        ebr_status st = validate_desc(desc);
        if (st) return st;
        Measured m;
        st = measure(desc, &m);
        if (st) return st;
        *arena_bytes = m.plan.total;
        return EBR_OK;
    } catch (const std::bad_alloc&) {
        set_error("host out of memory");
        return EBR_ENOMEM;
    } catch (...) {
        set_error("internal error");
        return EBR_EINVAL;
    }
}

ebr_status ebr_build_index(const ebr_build_desc* desc, void* dev_arena, size_t arena_bytes,
                           void* hip_stream, ebr_index** out) {
    try {
        if (!out) { set_error("out is NULL"); return EBR_EINVAL; }
        *out = nullptr;
        auto t0 = std::chrono::steady_clock::now();
        ebr_status st = validate_desc(desc);
        if (st) return st;
        Measured m;
        st = measure(desc, &m);
        if (st) return st;
        const ArenaPlan& p = m.plan;
        if (!dev_arena || arena_bytes < p.total) {
            set_error("arena too small: need %zu bytes, got %zu", p.total, arena_bytes);
            return EBR_ENOMEM;
        }
        if ((uintptr_t)dev_arena & 255) { set_error("arena must be 256-byte aligned"); return EBR_EINVAL; }
        const int64_t V = desc->n_keys;
        const int64_t n_post = V > 0 ? desc->key_offsets[V] : 0;

        // encode on the host
        std::vector<ChunkHdr> hdr((size_t)std::max<int64_t>(1, p.n_chunks));
        std::vector<uint32_t> words((size_t)p.n_words + 2, 0u);
        std::vector<float> maxw((size_t)V, 0.0f);
        if (V > 0) {
            parallel_for(V, [&](int64_t b, int64_t e) {
                for (int64_t k = b; k < e; ++k) {
                    const int64_t s = desc->key_offsets[k], t = desc->key_offsets[k + 1];
                    codec_encode(desc->post_ids + s, t - s, hdr.data() + m.key_chunk_off[k],
                                 words.data() + m.key_word_off[k], (uint32_t)m.key_word_off[k],
                                 (uint32_t)s);
                    float mx = (t > s) ? 1.0f : 0.0f;
                    if (desc->post_w) {
                        mx = 0.0f;
                        for (int64_t i = s; i < t; ++i) mx = std::max(mx, std::fabs(desc->post_w[i]));
                    }
                    maxw[k] = mx;
                }
            }, 256);
        }
        std::vector<float> emb(p.bytes_emb_f32 / 4);
        swizzle_f32(desc->ad_emb, desc->n_ads, desc->dim, emb.data());
        // reduced-precision copies and their error summaries
        const bool want_bf16 = desc->dtypes & (1u << EBR_BF16);
        const bool want_fp8 = desc->dtypes & (1u << EBR_FP8E4M3);
        std::vector<uint16_t> ebf((size_t)(want_bf16 ? p.bytes_emb_bf16 / 2 : 0), 0);
        std::vector<uint8_t> ef8((size_t)(want_fp8 ? p.bytes_emb_fp8 : 0), 0);
        std::vector<float> escale((size_t)(want_fp8 ? p.bytes_fp8_scale / 4 : 0), 1.0f);
        double q_err2[2] = {0, 0}, q_norm2[2] = {0, 0}, e_norm2 = 0;
        {
            const int d = desc->dim;
            const int nt = host_threads();
            std::vector<double> t_err[2], t_norm[2], t_e(nt, 0.0);
            for (int c = 0; c < 2; ++c) { t_err[c].assign(nt, 0.0); t_norm[c].assign(nt, 0.0); }
            std::vector<std::thread> th;
            const int64_t per = (desc->n_ads + nt - 1) / nt;
            for (int t = 0; t < nt; ++t) {
                th.emplace_back([&, t]() {
                    const int64_t b = t * per, e = std::min<int64_t>(desc->n_ads, b + per);
                    for (int64_t a = b; a < e; ++a) {
                        const float* row = desc->ad_emb + a * d;
                        double n2 = 0.0, mx = 0.0;
                        for (int k = 0; k < d; ++k) {
                            n2 += (double)row[k] * row[k];
                            mx = std::max(mx, std::fabs((double)row[k]));
                        }
                        t_e[t] = std::max(t_e[t], std::sqrt(n2));
                        if (want_bf16) {
                            double er = 0.0, nr = 0.0;
                            for (int k = 0; k < d; ++k) {
                                const uint16_t h = bf16_rne(row[k]);
                                ebf[mfma16_index(a, k, d)] = h;
                                const double q = bf16_to_f32(h);
                                er += (q - row[k]) * (q - row[k]);
                                nr += q * q;
                            }
                            t_err[0][t] = std::max(t_err[0][t], std::sqrt(er));
                            t_norm[0][t] = std::max(t_norm[0][t], std::sqrt(nr));
                        }
                        if (want_fp8) {
                            const float sc = mx > 0.0 ? (float)(mx / 448.0) : 1.0f;
                            escale[a] = sc;
                            double er = 0.0, nr = 0.0;
                            for (int k = 0; k < d; ++k) {
                                const uint8_t c8 = fp8_e4m3_rne(row[k] / sc);
                                ef8[mfma16_index(a, k, d)] = c8;
                                const double q = (double)sc * fp8_e4m3_to_f32(c8);
                                er += (q - row[k]) * (q - row[k]);
                                nr += q * q;
                            }
                            t_err[1][t] = std::max(t_err[1][t], std::sqrt(er));
                            t_norm[1][t] = std::max(t_norm[1][t], std::sqrt(nr));
                        }
                    }
                });
            }
            for (auto& x : th) x.join();
            for (int t = 0; t < nt; ++t) {
                e_norm2 = std::max(e_norm2, t_e[t]);
                for (int c = 0; c < 2; ++c) {
                    q_err2[c] = std::max(q_err2[c], t_err[c][t]);
                    q_norm2[c] = std::max(q_norm2[c], t_norm[c][t]);
                }
            }
        }
        const double enc_ms = ms_since(t0);

        // upload
        auto t1 = std::chrono::steady_clock::now();
        hipStream_t stream = (hipStream_t)hip_stream;
        char* base = (char*)dev_arena;
        HIP_TRY(hipMemcpyAsync(base + p.off_emb_f32, emb.data(), p.bytes_emb_f32, hipMemcpyHostToDevice, stream));
        if (want_bf16)
            HIP_TRY(hipMemcpyAsync(base + p.off_emb_bf16, ebf.data(), p.bytes_emb_bf16, hipMemcpyHostToDevice, stream));
        if (want_fp8) {
            HIP_TRY(hipMemcpyAsync(base + p.off_emb_fp8, ef8.data(), p.bytes_emb_fp8, hipMemcpyHostToDevice, stream));
            HIP_TRY(hipMemcpyAsync(base + p.off_fp8_scale, escale.data(), p.bytes_fp8_scale, hipMemcpyHostToDevice, stream));
        }
        if (p.n_chunks > 0)
            HIP_TRY(hipMemcpyAsync(base + p.off_chunks, hdr.data(), (size_t)p.n_chunks * 16, hipMemcpyHostToDevice, stream));
        HIP_TRY(hipMemcpyAsync(base + p.off_words, words.data(), p.bytes_words, hipMemcpyHostToDevice, stream));
        if (n_post > 0 && desc->post_w)
            HIP_TRY(hipMemcpyAsync(base + p.off_weights, desc->post_w, (size_t)n_post * 4,
                                   hipMemcpyHostToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        const double up_ms = ms_since(t1);

        ebr_index* ix = finish_index(desc->n_ads, desc->dim, desc->dtypes, V, n_post, desc->post_w != nullptr, p, base,
                                     std::move(m.key_chunk_off), desc->key_offsets, std::move(maxw), q_err2, q_norm2,
                                     e_norm2, enc_ms, up_ms);
        *out = ix;
        return EBR_OK;
    } catch (const std::bad_alloc&) {
        set_error("host out of memory");
        return EBR_ENOMEM;
    }
}


ebr_status ebr_device_build_scratch_size(int64_t n_keys, int64_t n_postings, size_t* bytes) {
    if (!bytes || n_keys < 0 || n_postings < 0) { set_error("bad argument"); return EBR_EINVAL; }
    *bytes = build_scratch(n_keys, n_postings).total;
    return EBR_OK;
}

ebr_status ebr_device_index_size(const ebr_build_desc* desc, void* scratch, size_t scratch_bytes, void* hip_stream,
                                 size_t* arena_bytes) {
    try {
        if (!arena_bytes) { set_error("arena_bytes is NULL"); return EBR_EINVAL; }
        BuildArgs a;
        std::vector<int64_t> ko;
        int64_t nc = 0, nw = 0;
        ebr_status st = device_shapes(desc, (char*)scratch, scratch_bytes, (hipStream_t)hip_stream, &a, &ko, &nc, &nw);
        if (st) return st;
        *arena_bytes = arena_plan(desc->n_ads, desc->dim, desc->dtypes, ko.back(), nc, nw, desc->post_w != nullptr).total;
        return EBR_OK;
    } catch (const std::bad_alloc&) {
        set_error("host out of memory");
        return EBR_ENOMEM;
    }
}

ebr_status ebr_build_index_device(const ebr_build_desc* desc, void* scratch, size_t scratch_bytes, void* dev_arena,
                                  size_t arena_bytes, void* hip_stream, ebr_index** out) {
    try {
        if (!out) { set_error("out is NULL"); return EBR_EINVAL; }
        *out = nullptr;
        const auto t0 = std::chrono::steady_clock::now();
        hipStream_t st = (hipStream_t)hip_stream;
        BuildArgs a;
        std::vector<int64_t> ko;
        int64_t nc = 0, nw = 0;
        ebr_status s = device_shapes(desc, (char*)scratch, scratch_bytes, st, &a, &ko, &nc, &nw);
        if (s) return s;
        const int64_t V = desc->n_keys, n_post = ko.back();
        const ArenaPlan p = arena_plan(desc->n_ads, desc->dim, desc->dtypes, n_post, nc, nw, desc->post_w != nullptr);
        if (!dev_arena || arena_bytes < p.total) { set_error("arena too small: need %zu bytes, got %zu", p.total, arena_bytes); return EBR_ENOMEM; }
        if ((uintptr_t)dev_arena & 255) { set_error("arena must be 256-byte aligned"); return EBR_EINVAL; }
        char* base = (char*)dev_arena;
        a.hdr = (ChunkHdr*)(base + p.off_chunks);
        a.words = (uint32_t*)(base + p.off_words);
        a.emb_f32 = (float*)(base + p.off_emb_f32);
        a.emb_bf16 = (desc->dtypes & (1u << EBR_BF16)) ? (uint16_t*)(base + p.off_emb_bf16) : nullptr;
        a.emb_fp8 = (desc->dtypes & (1u << EBR_FP8E4M3)) ? (uint8_t*)(base + p.off_emb_fp8) : nullptr;
        a.fp8_scale = a.emb_fp8 ? (float*)(base + p.off_fp8_scale) : nullptr;
        // rows first: non-finite embeddings are refused before the copies are written
        LAUNCH(launch_build_rows(a, st));
        unsigned long long flags[2] = {0, 0}, stats[5] = {0, 0, 0, 0, 0};
        HIP_TRY(hipMemcpyAsync(flags, a.flags, 16, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (flags[1] != ~0ull) { set_error("non-finite embedding in ad %llu", flags[1]); return EBR_EINVAL; }
        LAUNCH(launch_build_pack(a, st));
        LAUNCH(launch_fill_u32(a.words + nw, 0u, 2, st));  // the two pad words
        LAUNCH(launch_build_layout(a, st));
        if (desc->post_w && n_post > 0)
            HIP_TRY(hipMemcpyAsync(base + p.off_weights, desc->post_w, 4 * (size_t)n_post, hipMemcpyDeviceToDevice, st));
        std::vector<uint32_t> kco((size_t)V + 1, 0u);
        std::vector<float> maxw((size_t)V, 0.0f);
        HIP_TRY(hipMemcpyAsync(stats, a.stats, 40, hipMemcpyDeviceToHost, st));
        if (V > 0) {
            HIP_TRY(hipMemcpyAsync(kco.data(), a.key_chunk_off, 4 * (size_t)(V + 1), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(maxw.data(), a.key_maxw, 4 * (size_t)V, hipMemcpyDeviceToHost, st));
        }
        HIP_TRY(hipStreamSynchronize(st));
        auto root = [&](int i) {
            double v;
            std::memcpy(&v, &stats[i], 8);
            return std::sqrt(v);  // the largest row norm: the root of the largest squared norm
        };
        const double q_err2[2] = {root(1), root(3)}, q_norm2[2] = {root(2), root(4)};
        *out = finish_index(desc->n_ads, desc->dim, desc->dtypes, V, n_post, desc->post_w != nullptr, p, base,
                            std::move(kco), ko.data(), std::move(maxw), q_err2, q_norm2, root(0), ms_since(t0), 0.0);
        return EBR_OK;
    } catch (const std::bad_alloc&) {
        set_error("host out of memory");
        return EBR_ENOMEM;
    }
}

ebr_status ebr_index_stats(const ebr_index* index, ebr_index_info* out) {
    if (!index || !out) { set_error("NULL argument"); return EBR_EINVAL; }
    *out = index->stats;
    return EBR_OK;
}

void ebr_free_index(ebr_index* index) { delete index; }

ebr_status ebr_decode_keys(const ebr_index* index, int64_t key_begin, int64_t key_end, uint32_t* ids,
                           float* w, int64_t cap, int64_t* len, void* hip_stream) {
    if (!index || !len) { set_error("NULL argument"); return EBR_EINVAL; }
    if (key_begin < 0 || key_end < key_begin || key_end > index->n_keys) {
        set_error("key range [%lld, %lld) outside [0, %lld)", (long long)key_begin, (long long)key_end,
                  (long long)index->n_keys);
        return EBR_EINVAL;
    }
    const int64_t p0 = index->key_post_off[key_begin], n = index->key_post_off[key_end] - p0;
    *len = n;
    if (cap < n) { set_error("capacity %lld < %lld postings", (long long)cap, (long long)n); return EBR_ENOMEM; }
    if (n == 0) return EBR_OK;
    if (!ids || !w) { set_error("NULL output"); return EBR_EINVAL; }
    const uint32_t c0 = index->key_chunk_off[key_begin], c1 = index->key_chunk_off[key_end];
    int rc = launch_decode_key(index->chunks, index->words, index->weights, c0, c1 - c0, (uint32_t)p0,
                               ids, w, hip_stream);
    if (rc) { set_error("decode launch failed: %s", hipGetErrorString((hipError_t)rc)); return EBR_EDEVICE; }
    HIP_TRY(hipStreamSynchronize((hipStream_t)hip_stream));
    return EBR_OK;
}

ebr_status ebr_decode_key(const ebr_index* index, int64_t key, uint32_t* ids, float* w,
                          int64_t cap, int64_t* len, void* hip_stream) {
    if (index && (key < 0 || key >= index->n_keys)) { set_error("key %lld out of range", (long long)key); return EBR_EINVAL; }
    return ebr_decode_keys(index, key, key + 1, ids, w, cap, len, hip_stream);
}

}  // extern "C"

// ====================================================================== batch planning

namespace ebr {

struct Plan {
    int dtype = 0;        // scan copy: 0 FP32, 1 BF16, 2 FP8
    bool w64 = false;     // 64-bit cross-term cells (FP32 scan, 128-query groups)
    int factor = 1;       // approximate scans: candidates rescored per result
    int B = 0, gq = 256, n_qg = 0, nu = 0;
    std::vector<int32_t> kcnt;  // per query: K (FP32 scan) or K' = min(N, factor K)
    int kcmax = 0;
    std::vector<double> aq;     // per query: sum_j |m_j| max|W[k_j,:]|
    bool packed = false;  // bucket entries carry users ranges: one query group, < 2^19 features
    bool split = false;   // split buckets (several query groups, see kernels.h)
    int n_sub = 1, n_hot = 0, cold_first = 0;
    std::vector<uint32_t> hot_tab, hot_users, hot_users_off, cold_off, cold_users;
    int64_t nnz = 0;
    int kmax = 0;
    std::vector<uint32_t> uk_chunk_begin, uk_chunk_prefix, users_off, users;
    std::vector<int32_t> uk_wshift;
    std::vector<double> qinv;
    std::vector<float> werr;    // per query: F_q / 2 quanta, the cross term's rounding bound
    std::vector<int32_t> kq, jq;  // kq: K of the selection path (0 for full-sort queries)
    std::vector<int32_t> big;     // queries answered by a full sort (K beyond the LDS sort)
    std::vector<int64_t> out_off;
    std::vector<uint32_t> sample_tiles;
    int64_t n_sample_valid = 0;
    uint64_t bucket_n = 0;
    uint32_t total_chunks = 0;
    int64_t n_tiles = 0;
    // workspace layout
    size_t off_plan = 0, plan_bytes = 0;
    size_t o_kc = 0, o_aq = 0, off_ctl = 0, off_cwide = 0, off_rid = 0, off_rwide = 0, off_rst = 0, off_eps = 0,
           off_unc = 0, off_fb_users = 0, off_fb_ids = 0, off_fb_scores = 0, fb_limit = 0;
    size_t o_ukb = 0, o_ukp = 0, o_ukw = 0, o_uoff = 0, o_users = 0, o_qi = 0, o_kq = 0, o_jq = 0,
           o_oo = 0, o_st = 0, o_werr = 0, o_htab = 0, o_husers = 0, o_hoff = 0, o_coff = 0,
           o_cusers = 0;
    int64_t n_super = 0;
    int sshift = kSuperShift;  // log2 of the ads per decode super-tile
    size_t off_stcnt = 0, off_stoff = 0, off_stfill = 0, off_stage = 0, off_cmap = 0;
    size_t off_big_deep = 0, off_big_wide = 0, off_big_keys = 0, off_big_tmp = 0, off_big_hist = 0,
           off_big_stmp = 0;
    size_t off_toff = 0, off_stmp = 0, off_bucket = 0, off_skeys = 0,
           off_thr = 0, off_status = 0, off_active = 0, off_ccnt = 0, off_unres = 0, off_cand = 0;
    size_t total = 0;
};

// Per-thread planner scratch sized to the key space: a slot per key (distinct keys of a batch;
// all -1 between calls).
struct PlanScratch {
    std::vector<int32_t> slot_of;
};

static PlanScratch& plan_scratch(int64_t n_keys) {
    static thread_local PlanScratch ps;
    if ((int64_t)ps.slot_of.size() < n_keys) ps.slot_of.assign((size_t)n_keys, -1);
    return ps;
}

// Sample tiles of the threshold pre-pass: at least n_tiles / 128 tiles and 16 K' ads.
static int64_t sample_tile_count(const Index& ix, int kcmax) {
    const int64_t nt = ix.n_tiles;
    const int64_t ns = std::max<int64_t>((nt + 127) / 128, (16LL * kcmax + kTileAds - 1) / kTileAds);
    return std::min(ns, nt);
}

static size_t layout_total(const Index& ix, const BatchSizes& z, int dtype, bool w64);

// Workspace sections of one batch; depends only on the batch's sizes (and the scan dtype and
// cell width, which P holds on entry along with the query-group size).
static void layout(const Index& ix, bool topk, const BatchSizes& z, Plan* P) {
    const int B = z.B;
    const int nu = z.nu;
    const int nqg = std::max(1, (B + P->gq - 1) / P->gq);
    const size_t n_users_off = (size_t)nu * nqg + 1, n_users = 2 * (size_t)std::max<int64_t>(1, z.nnz);
    P->bucket_n = z.bucket_n;
    const bool split = split_groups(nqg) && nu < (1 << 21);
    P->n_sub = split ? nqg + 2 : 1;
    size_t off = 0;
    auto put = [&](size_t bytes) { size_t o = off; off = align256(off + std::max<size_t>(bytes, 16)); return o; };
    P->off_plan = off;
    P->o_ukb = put(4 * (size_t)nu);
    P->o_ukp = put(4 * (size_t)(nu + 1));
    P->o_ukw = put(4 * (size_t)nu);
    P->o_uoff = put(4 * n_users_off);
    P->o_users = put(4 * n_users);
    P->o_qi = put(8 * (size_t)B);
    P->o_kq = put(4 * (size_t)B);
    P->o_jq = put(4 * (size_t)B);
    P->o_kc = put(4 * (size_t)B);
    P->o_aq = put(8 * (size_t)B);
    P->o_werr = put(4 * (size_t)B);
    P->o_oo = put(8 * (size_t)(B + 1));
    P->o_st = put(4 * (size_t)z.n_sample);
    if (split) {
        P->o_htab = put(4 * (size_t)nqg * (size_t)std::min(nu, kHotMax));
        P->o_husers = put(4 * n_users);
        P->o_hoff = put(4 * (size_t)(nqg + 1));
        P->o_coff = put(4 * (size_t)(nu + 1));
        P->o_cusers = put(4 * n_users);
    }
    P->plan_bytes = off - P->off_plan;
    // super-tiles of the list decode: 2048 ads without split buckets (longer runs of a list's
    // postings per super-tile, so fewer atomics and longer writes; measured best of 1024..8192
    // ads on 256-query batches) when the slots fit the entry's bits, else 1024; the counters
    // are sized for 1024-ad super-tiles either way, so that a rerun subset of the batch, which
    // may take the other size, fits the layout
    const int64_t n_super_max = (ix.n_ads + kSuperAds - 1) / kSuperAds;
    P->sshift = (!split && z.nu < (1 << (32 - kMaxSuperShift))) ? kMaxSuperShift : kSuperShift;
    P->n_super = (ix.n_ads + (1LL << P->sshift) - 1) >> P->sshift;
    P->off_stcnt = put(4 * (size_t)(n_super_max + 1));
    P->off_stoff = put(4 * (size_t)(n_super_max + 1));
    P->off_stfill = put(4 * (size_t)(n_super_max + 1));
    P->off_stmp = put(4 * (size_t)scan_tmp_words(n_super_max + 1));
    P->off_stage = put(8 * (size_t)P->bucket_n);
    // chunks of the batch: sum over keys of ceil(L / 64) <= postings / 64 + keys
    P->off_cmap = put(8 * ((size_t)P->bucket_n / kChunk + (size_t)nu + 1));
    P->off_toff = put(4 * (size_t)(ix.n_tiles * P->n_sub + 1));
    P->off_bucket = put(8 * (size_t)P->bucket_n);
    if (topk) {
        P->off_skeys = put(4 * (size_t)B * (size_t)z.n_sample * kTileAds);
        P->off_thr = put(8 * (size_t)B);
        P->off_status = put(4 * (size_t)B);
        P->off_active = put(4 * (size_t)B);
        P->off_ccnt = put(4 * (size_t)B);
        P->off_unres = put(16);
        P->off_ctl = put(sizeof(Control));
        P->off_cand = put(8 * (size_t)B * kCandCap);
        if (P->dtype != EBR_F32) {
            P->off_cwide = put(4 * (size_t)B * kCandCap);
            P->off_rid = put(4 * (size_t)B * std::max(1, z.kcmax));
            P->off_rwide = put(4 * (size_t)B * std::max(1, z.kcmax));
            P->off_rst = put(4 * (size_t)B);
            P->off_eps = put(4 * (size_t)B);
            P->off_unc = put(16);
        }
        if (!P->w64) {
            // rerun region: after the batch, a subset of its queries runs again in the bytes
            // below fb_limit, on the FP32 scan (failed recall certificates) or with 64-bit
            // cells (imprecise cross terms); the subset's users and results sit above it
            size_t sub = layout_total(ix, z, EBR_F32, true);
            if (P->dtype != EBR_F32) sub = std::max(sub, layout_total(ix, z, EBR_F32, false));
            off = align256(std::max(off, sub));
            P->fb_limit = off;
            P->off_fb_users = put(4 * (size_t)B * ix.dim);
            P->off_fb_ids = put(4 * (size_t)std::max<int64_t>(1, z.n_out));
            P->off_fb_scores = put(4 * (size_t)std::max<int64_t>(1, z.n_out));
        }
        if (z.big_n > 0) {
            // full sort of one query's scores (queries whose K exceeds the LDS sort); its dense
            // pass runs in the bytes below fb_limit (or the batch's own, 64-bit cells)
            const size_t n = (size_t)z.big_n, nb = (size_t)sort_blocks(z.big_n);
            P->off_big_deep = put(4 * n);
            P->off_big_wide = put(4 * n);
            P->off_big_keys = put(8 * n);
            P->off_big_tmp = put(8 * n);
            P->off_big_hist = put(4 * (256 * nb + 1));
            P->off_big_stmp = put(4 * (size_t)scan_tmp_words((int64_t)(256 * nb)));
        }
    }
    P->total = off;
}

// Total workspace of a top-K batch of sizes z on scan dtype `dtype` with 32- or 64-bit cells.
static size_t layout_total(const Index& ix, const BatchSizes& z, int dtype, bool w64) {
    Plan Q;
    Q.dtype = dtype;
    Q.w64 = w64;
    Q.gq = score_group_queries(ix.dim, w64);
    layout(ix, true, z, &Q);
    return Q.total;
}

static ebr_status plan_batch(const Index& ix, const ebr_batch* bt, bool topk, Plan* P) {
    if (!bt) { set_error("batch is NULL"); return EBR_EINVAL; }
    const int B = bt->n_queries;
    if (B < 0) { set_error("n_queries < 0"); return EBR_EINVAL; }
    if (bt->scan_dtype != EBR_F32 && bt->scan_dtype != EBR_BF16 && bt->scan_dtype != EBR_FP8E4M3) {
        set_error("unknown scan dtype %d", (int)bt->scan_dtype);
        return EBR_EINVAL;
    }
    P->dtype = (int)bt->scan_dtype;
    if ((P->dtype == EBR_BF16 && !ix.emb_bf16) || (P->dtype == EBR_FP8E4M3 && !ix.emb_fp8)) {
        set_error("the index holds no %s copy (build it with that dtype bit)",
                  P->dtype == EBR_BF16 ? "BF16" : "FP8");
        return EBR_EUNSUPPORTED;
    }
    if (bt->wide64 != 0 && bt->wide64 != 1) { set_error("wide64 must be 0 or 1"); return EBR_EINVAL; }
    P->w64 = bt->wide64 == 1;
    if (P->w64 && P->dtype != EBR_F32) { set_error("64-bit cross-term cells need the FP32 scan"); return EBR_EINVAL; }
    P->factor = P->dtype == EBR_F32 ? 1 : (bt->rescore_factor > 0 ? bt->rescore_factor : 4);
    P->B = B;
    P->gq = score_group_queries(ix.dim, P->w64);
    P->n_qg = (B + P->gq - 1) / P->gq;
    P->n_tiles = ix.n_tiles;
    if (B > 0 && (!bt->user_emb || !bt->feat_offsets || (topk && !bt->k))) { set_error("NULL batch array"); return EBR_EINVAL; }
    const int64_t nnz = B > 0 ? bt->feat_offsets[B] : 0;
    if (B > 0 && bt->feat_offsets[0] != 0) { set_error("feat_offsets[0] != 0"); return EBR_EINVAL; }
    for (int q = 0; q < B; ++q)
        if (bt->feat_offsets[q + 1] < bt->feat_offsets[q]) { set_error("feat_offsets decrease at query %d", q); return EBR_EINVAL; }
    if (nnz > 0 && !bt->feat_keys) { set_error("feat_keys is NULL"); return EBR_EINVAL; }
    P->nnz = nnz;
    if (nnz >= (1LL << 31)) { set_error("more than 2^31 features in one batch"); return EBR_EINVAL; }
    // keys in range, distinct within a query, multipliers finite; and the distinct keys of
    // the batch, in order of first use, with each feature's key slot (one pass: a key's slot,
    // then the last query that used the slot)
    PlanScratch& ps = plan_scratch(ix.n_keys);
    std::vector<int32_t> uk;
    std::vector<int32_t> slot(nnz);
    {
        std::vector<int32_t> last_q;
        auto undo = [&]() { for (int32_t k : uk) ps.slot_of[k] = -1; };
        for (int q = 0; q < B; ++q) {
            const int64_t f0 = bt->feat_offsets[q], f1 = bt->feat_offsets[q + 1];
            for (int64_t j = f0; j < f1; ++j) {
                const int32_t k = bt->feat_keys[j];
                if (k < 0 || k >= ix.n_keys) {
                    undo();
                    set_error("query %d: key %d out of range [0, %lld)", q, k, (long long)ix.n_keys);
                    return EBR_EINVAL;
                }
                int32_t sl = ps.slot_of[k];
                if (sl < 0) {
                    sl = (int32_t)uk.size();
                    ps.slot_of[k] = sl;
                    uk.push_back(k);
                    last_q.push_back(-1);
                }
                if (last_q[sl] == q) { undo(); set_error("query %d repeats a key", q); return EBR_EINVAL; }
                last_q[sl] = q;
                slot[j] = sl;
            }
            if (bt->feat_mult)
                for (int64_t j = f0; j < f1; ++j)
                    if (!std::isfinite(bt->feat_mult[j])) { undo(); set_error("query %d: non-finite multiplier", q); return EBR_EINVAL; }
        }
        undo();
    }
    P->kq.assign(B, 0);
    P->kmax = 0;
    P->big.clear();
    std::vector<int64_t> ktrue(B, 0);
    if (topk) {
        for (int q = 0; q < B; ++q) {
            if (bt->k[q] < 0 || (int64_t)bt->k[q] > ix.n_ads) { set_error("query %d: K = %d outside [0, %lld]", q, bt->k[q], (long long)ix.n_ads); return EBR_EINVAL; }
            ktrue[q] = bt->k[q];
            // candidates beyond the LDS sort of the selection path: answered by a full sort
            const int64_t kc = std::min<int64_t>(ix.n_ads, (int64_t)P->factor * bt->k[q]);
            if (kc > kMaxK) { P->big.push_back(q); continue; }
            P->kq[q] = bt->k[q];
            P->kmax = std::max(P->kmax, bt->k[q]);
        }
    }
    P->kcnt.assign(B, 0);
    P->kcmax = 0;
    for (int q = 0; q < B; ++q) {
        const int64_t kc = P->kq[q] == 0 ? 0 : std::min<int64_t>(ix.n_ads, (int64_t)P->factor * P->kq[q]);
        P->kcnt[q] = (int32_t)kc;
        P->kcmax = std::max(P->kcmax, (int)kc);
    }
    const int nu = (int)uk.size();
    if (nu >= (1 << (32 - kSuperShift))) { set_error("too many distinct keys in one batch"); return EBR_EINVAL; }
    P->nu = nu;
    P->packed = P->n_qg == 1 && nnz < (1LL << 19);
    // split buckets (several query groups): hot keys first, then warm, then cold (kernels.h)
    const int nqg = std::max(1, P->n_qg);
    P->split = split_groups(nqg) && nu < (1 << 21);
    P->n_sub = P->split ? nqg + 2 : 1;
    P->n_hot = 0;
    P->cold_first = nu;
    std::vector<uint32_t> ucnt;  // split: users per slot (all groups)
    if (P->split) {
        std::vector<uint32_t> users_of(nu, 0u);
        for (int64_t j = 0; j < nnz; ++j) users_of[slot[j]]++;
        // cold: at most as many users as groups (placing a posting once per user costs less
        // than every group visiting it); hot: of the others, the longest lists first (ties by
        // slot), while each group's users of them fit its LDS records; warm: the rest
        const uint32_t limit = (uint32_t)cold_user_limit(nqg);
        std::vector<uint64_t> by_len;  // (~length << 32) | slot of the non-cold keys, ascending
        std::vector<int32_t> cand(nu, -1);
        for (int u = 0; u < nu; ++u)
            if (users_of[u] > limit) {
                cand[u] = (int32_t)by_len.size();
                const uint64_t L = (uint64_t)(ix.key_post_off[uk[u] + 1] - ix.key_post_off[uk[u]]);
                by_len.push_back(((~L & 0xffffffffull) << 32) | (uint64_t)u);
            }
        // per (non-cold key, group): users
        std::vector<uint32_t> cnt(by_len.size() * (size_t)nqg, 0u);
        parallel_for(nqg, [&](int64_t g0, int64_t g1) {  // a group's queries touch its column only
            for (int64_t g = g0; g < g1; ++g) {
                const int q1 = std::min(B, (int)(g + 1) * P->gq);
                for (int q = (int)g * P->gq; q < q1; ++q)
                    for (int64_t j = bt->feat_offsets[q]; j < bt->feat_offsets[q + 1]; ++j)
                        if (cand[slot[j]] >= 0) cnt[(size_t)cand[slot[j]] * nqg + g]++;
            }
        }, 1);
        std::sort(by_len.begin(), by_len.end());
        const uint32_t cap = (uint32_t)score_users_lds(ix.dim, P->w64);
        std::vector<uint32_t> hu(nqg, 0u);
        std::vector<int32_t> order;
        order.reserve(nu);
        for (uint64_t key : by_len) {
            const int32_t u = (int32_t)(key & 0xffffffffu);
            if ((int)order.size() == kHotMax) break;
            const uint32_t* c = cnt.data() + (size_t)cand[u] * nqg;
            bool fits = true;
            for (int g = 0; g < nqg && fits; ++g) fits = hu[g] + c[g] <= cap;
            if (!fits) continue;
            for (int g = 0; g < nqg; ++g) hu[g] += c[g];
            order.push_back(u);
        }
        std::vector<char> is_hot(nu, 0);
        for (int32_t u : order) is_hot[u] = 1;
        P->n_hot = (int)order.size();
        for (int u = 0; u < nu; ++u)
            if (!is_hot[u] && users_of[u] > limit) order.push_back(u);
        P->cold_first = (int)order.size();
        for (int u = 0; u < nu; ++u)
            if (!is_hot[u] && users_of[u] <= limit) order.push_back(u);
        // renumber the slots in that order
        std::vector<int32_t> renum(nu);
        std::vector<int32_t> uk2(nu);
        ucnt.resize(nu);
        for (int i = 0; i < nu; ++i) {
            renum[order[i]] = i;
            uk2[i] = uk[order[i]];
            ucnt[i] = users_of[order[i]];
        }
        uk.swap(uk2);
        for (int64_t j = 0; j < nnz; ++j) slot[j] = renum[slot[j]];
    }
    P->uk_chunk_begin.resize(nu);
    P->uk_chunk_prefix.assign(nu + 1, 0);
    P->uk_wshift.resize(nu);
    uint64_t chunks = 0, posts = 0;
    for (int u = 0; u < nu; ++u) {
        const int k = uk[u];
        P->uk_chunk_begin[u] = ix.key_chunk_off[k];
        P->uk_chunk_prefix[u] = (uint32_t)chunks;
        P->uk_wshift[u] = ix.key_wshift[k];
        chunks += ix.key_chunk_off[k + 1] - ix.key_chunk_off[k];
        posts += (uint64_t)(ix.key_post_off[k + 1] - ix.key_post_off[k]);
    }
    P->uk_chunk_prefix[nu] = (uint32_t)chunks;
    P->total_chunks = (uint32_t)chunks;
    P->bucket_n = posts;
    if (P->split) {
        // a cold key's postings are placed once per user
        for (int u = P->cold_first; u < nu; ++u)
            P->bucket_n += (uint64_t)(ix.key_post_off[uk[u] + 1] - ix.key_post_off[uk[u]]) * (ucnt[u] - 1u);
    }
    // users of each (distinct key, query group), in query order; the groups' entries are
    // disjoint, so groups are counted and filled in parallel
    auto per_group = [&](const std::function<void(int)>& fn) {
        parallel_for(nqg, [&](int64_t g0, int64_t g1) { for (int64_t g = g0; g < g1; ++g) fn((int)g); }, 1);
    };
    P->users_off.assign((size_t)nu * nqg + 1, 0);
    per_group([&](int g) {
        const int q1 = std::min(B, (g + 1) * P->gq);
        for (int q = g * P->gq; q < q1; ++q)
            for (int64_t j = bt->feat_offsets[q]; j < bt->feat_offsets[q + 1]; ++j)
                P->users_off[(size_t)slot[j] * nqg + g + 1]++;
    });
    {
        // inclusive prefix of users_off in place: per-slice sums, their prefix, then each slice
        std::vector<uint32_t>& uo = P->users_off;
        const int64_t n = (int64_t)uo.size();
        const int ns = n > (1 << 18) ? 16 : 1;
        const int64_t per = (n + ns - 1) / ns;
        std::vector<uint32_t> part(ns + 1, 0u);
        parallel_for(ns, [&](int64_t t0, int64_t t1) {
            for (int64_t t = t0; t < t1; ++t) {
                uint32_t acc = 0;
                for (int64_t i = t * per, e = std::min(n, (t + 1) * per); i < e; ++i) acc += uo[(size_t)i];
                part[(size_t)t + 1] = acc;
            }
        }, 1);
        for (int t = 0; t < ns; ++t) part[(size_t)t + 1] += part[(size_t)t];
        parallel_for(ns, [&](int64_t t0, int64_t t1) {
            for (int64_t t = t0; t < t1; ++t) {
                uint32_t acc = part[(size_t)t];
                for (int64_t i = t * per, e = std::min(n, (t + 1) * per); i < e; ++i) uo[(size_t)i] = acc += uo[(size_t)i];
            }
        }, 1);
    }
    // per-query fixed-point scale of the cross term: the largest S with
    // sum_j |m_j| max|W[k_j,:]| 2^S (1 + 2^-23) + F_q + 1 below 2^31 (2^63 for 64-bit cells), so
    // that every (query, ad) sum of rounded terms fits the cell; a sum's rounding error is at
    // most F_q / 2 quanta of 2^-S
    std::vector<int> Sq(B, 0);
    P->qinv.assign(B, 1.0);
    P->aq.assign(B, 0.0);
    P->werr.assign(B, 0.0f);
    const int cell_bits = P->w64 ? 63 : 31;
    parallel_for(B, [&](int64_t q0, int64_t q1) { for (int64_t q = q0; q < q1; ++q) {
        double A = 0.0;
        const int64_t F = bt->feat_offsets[q + 1] - bt->feat_offsets[q];
        for (int64_t j = bt->feat_offsets[q]; j < bt->feat_offsets[q + 1]; ++j) {
            const double m = bt->feat_mult ? (double)bt->feat_mult[j] : 1.0;
            A += std::fabs(m) * (double)ix.key_maxw[bt->feat_keys[j]];
        }
        P->aq[q] = A;
        int S = 0;
        if (A > 0.0 && std::isfinite(A)) {
            int e;
            std::frexp(A, &e);  // A < 2^e
            S = cell_bits - e;
            if (std::ldexp(A, S) * (1.0 + 0x1p-23) + (double)F + 1.0 >= std::ldexp(1.0, cell_bits)) --S;
            S = std::max(-126, std::min(126, S));
        }
        Sq[q] = S;
        P->qinv[q] = std::ldexp(1.0, -S);
        P->werr[q] = (float)std::ldexp((double)F, -S - 1);
    } }, nnz > (1 << 16) ? 64 : std::max(B, 1));  // small batches: one thread (waking the pool costs more)
    // users: (query within its group, bits of m' = m * 2^(S_q - Sw_k) in FP32), in query order;
    // |m'| <= 2^(e(max|W_k|) - e(A_q) + 1) |m| max|W_k| / max|W_k| stays far from overflow
    P->users.assign((size_t)2 * std::max<int64_t>(1, nnz), 0u);
    {
        std::vector<uint32_t> fill(P->users_off.begin(), P->users_off.end() - 1);
        per_group([&](int g) {
            const int q1 = std::min(B, (g + 1) * P->gq);
            for (int q = g * P->gq; q < q1; ++q)
                for (int64_t j = bt->feat_offsets[q]; j < bt->feat_offsets[q + 1]; ++j) {
                    const uint32_t pos = fill[(size_t)slot[j] * nqg + g]++;
                    const double m = bt->feat_mult ? (double)bt->feat_mult[j] : 1.0;
                    const int sw = ix.key_wshift[bt->feat_keys[j]];
                    const float mf = (float)std::ldexp(m, Sq[q] - sw);
                    uint32_t bits;
                    std::memcpy(&bits, &mf, 4);
                    P->users[2 * pos] = (uint32_t)(q - g * P->gq);
                    P->users[2 * pos + 1] = bits;
                }
        });
    }
    if (P->split) {
        // per group: its users of the hot keys (the LDS records of its work-groups) and the
        // table hot slot -> (first record << 9) | count
        const int H = P->n_hot;
        P->hot_tab.assign((size_t)nqg * std::max(1, H), 0u);
        P->hot_users_off.assign(nqg + 1, 0u);
        for (int g = 0; g < nqg; ++g) {
            uint32_t n = 0;
            for (int u = 0; u < H; ++u) n += P->users_off[(size_t)u * nqg + g + 1] - P->users_off[(size_t)u * nqg + g];
            P->hot_users_off[g + 1] = P->hot_users_off[g] + n;
        }
        P->hot_users.assign(2 * (size_t)std::max(1u, P->hot_users_off[nqg]), 0u);
        per_group([&](int g) {
            uint32_t local = 0;
            uint32_t* dst = P->hot_users.data() + 2 * (size_t)P->hot_users_off[g];
            for (int u = 0; u < H; ++u) {
                const uint32_t b = P->users_off[(size_t)u * nqg + g], e = P->users_off[(size_t)u * nqg + g + 1];
                P->hot_tab[(size_t)g * H + u] = (local << 9) | (e - b);
                std::memcpy(dst + 2 * (size_t)local, P->users.data() + 2 * (size_t)b, 8 * (size_t)(e - b));
                local += e - b;
            }
        });
        // per cold key: its users of all groups as (query index in the batch, m'); a key's
        // users of all groups are contiguous in users (slot-major offsets)
        const int nc = nu - P->cold_first;
        P->cold_off.assign((size_t)nc + 1, 0u);
        for (int c = 0; c < nc; ++c) {
            const size_t u = (size_t)(P->cold_first + c);
            P->cold_off[c + 1] = P->cold_off[c] + (P->users_off[(u + 1) * nqg] - P->users_off[u * nqg]);
        }
        P->cold_users.assign(2 * (size_t)std::max(1u, P->cold_off[nc]), 0u);
        parallel_for(nc, [&](int64_t c0, int64_t c1) {
            for (int64_t c = c0; c < c1; ++c) {
                const size_t u = (size_t)(P->cold_first + c);
                uint32_t* dst = P->cold_users.data() + 2 * (size_t)P->cold_off[c];
                for (int g = 0; g < nqg; ++g)
                    for (uint32_t i = P->users_off[u * nqg + g]; i < P->users_off[u * nqg + g + 1]; ++i) {
                        *dst++ = (uint32_t)g * (uint32_t)P->gq + P->users[2 * (size_t)i];
                        *dst++ = P->users[2 * (size_t)i + 1];
                    }
            }
        }, 8192);
    }
    // the kernel reads each user's row as its cell code (acc_row_code); the cold records
    // above keep the query index
    {
        const uint32_t n = P->users_off.back();
        parallel_for(n, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) P->users[2 * i] = acc_row_code(P->users[2 * i], P->w64);
        }, 1 << 16);
        const uint32_t nh = P->split ? P->hot_users_off[nqg] : 0u;
        parallel_for(nh, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) P->hot_users[2 * i] = acc_row_code(P->hot_users[2 * i], P->w64);
        }, 1 << 16);
    }
    // output offsets
    P->out_off.assign(B + 1, 0);
    for (int q = 0; q < B; ++q) P->out_off[q + 1] = P->out_off[q] + ktrue[q];
    // sample tiles for the threshold: spread evenly, at least n_tiles / 128 and 16 * K ads
    P->jq.assign(B, 0);
    P->sample_tiles.clear();
    if (topk && P->kmax > 0) {
        const int64_t nt = ix.n_tiles;
        const int64_t ns = sample_tile_count(ix, P->kcmax);
        P->sample_tiles.resize(ns);
        int64_t valid = 0;
        for (int64_t i = 0; i < ns; ++i) {
            const int64_t t = (i * nt) / ns;
            P->sample_tiles[i] = (uint32_t)t;
            valid += std::min<int64_t>(kTileAds, ix.n_ads - t * kTileAds);
        }
        P->n_sample_valid = valid;
        const double f = (double)valid / (double)ix.n_ads;
        for (int q = 0; q < B; ++q) {
            const int K = P->kcnt[q];
            if (K == 0) continue;
            if (ns == nt) { P->jq[q] = K; continue; }
            // x = K' f sample ads are expected among the K' best; j sits 5 standard deviations
            // (Poisson) above, so too few survivors (j - x > 5 sqrt(x)) is rarer than 1e-5; the
            // survivors, about j / f (at most ~12.5 K for K' <= 8192 with either sampling
            // rule), stay more than 4 standard deviations below the 16384-slot buffer
            const double x = K * f;
            int64_t j = (int64_t)std::ceil(x + 5.0 * std::sqrt(x) + 4.0);
            P->jq[q] = (int32_t)std::min<int64_t>(j, valid);
        }
    }
    BatchSizes z;
    z.B = B;
    z.nnz = nnz;
    z.nu = nu;
    z.bucket_n = P->bucket_n;
    z.kcmax = P->kcmax;
    z.n_out = P->out_off[B];
    z.n_sample = (int64_t)P->sample_tiles.size();
    z.big_n = P->big.empty() ? 0 : ix.n_ads;
    layout(ix, topk, z, P);
    return EBR_OK;
}

// The plan's arrays into dst (P.plan_bytes bytes: the workspace's plan section), copied in
// pieces of at most 1 MiB spread over the host threads; the bytes between the arrays
// (alignment padding, reserved space a batch leaves unused) are zeroed.
static void pack_plan_into(const Plan& P, char* dst) {
    struct Piece {
        size_t o;
        const void* src;
        size_t n;
    };
    std::vector<Piece> pcs;
    auto add = [&](size_t o, const void* src, size_t n) { if (n) pcs.push_back({o - P.off_plan, src, n}); };
    add(P.o_ukb, P.uk_chunk_begin.data(), 4 * P.uk_chunk_begin.size());
    add(P.o_ukp, P.uk_chunk_prefix.data(), 4 * P.uk_chunk_prefix.size());
    add(P.o_uoff, P.users_off.data(), 4 * P.users_off.size());
    add(P.o_users, P.users.data(), 4 * P.users.size());
    add(P.o_ukw, P.uk_wshift.data(), 4 * P.uk_wshift.size());
    add(P.o_qi, P.qinv.data(), 8 * P.qinv.size());
    add(P.o_kq, P.kq.data(), 4 * P.kq.size());
    add(P.o_jq, P.jq.data(), 4 * P.jq.size());
    add(P.o_kc, P.kcnt.data(), 4 * P.kcnt.size());
    add(P.o_aq, P.aq.data(), 8 * P.aq.size());
    add(P.o_werr, P.werr.data(), 4 * P.werr.size());
    add(P.o_oo, P.out_off.data(), 8 * P.out_off.size());
    add(P.o_st, P.sample_tiles.data(), 4 * P.sample_tiles.size());
    if (P.split) {
        add(P.o_htab, P.hot_tab.data(), 4 * (size_t)P.n_hot * (P.hot_users_off.size() - 1));
        add(P.o_husers, P.hot_users.data(), 4 * P.hot_users.size());
        add(P.o_hoff, P.hot_users_off.data(), 4 * P.hot_users_off.size());
        add(P.o_coff, P.cold_off.data(), 4 * P.cold_off.size());
        add(P.o_cusers, P.cold_users.data(), 4 * P.cold_users.size());
    }
    std::sort(pcs.begin(), pcs.end(), [](const Piece& a, const Piece& b) { return a.o < b.o; });
    std::vector<Piece> parts;
    size_t at = 0;
    static const char kZeros[4096] = {};
    auto zero = [&](size_t o, size_t n) {
        for (size_t b = 0; b < n; b += sizeof(kZeros)) parts.push_back({o + b, kZeros, std::min(sizeof(kZeros), n - b)});
    };
    constexpr size_t kPiece = 1 << 20;
    for (const Piece& p : pcs) {
        if (p.o > at) zero(at, p.o - at);
        for (size_t b = 0; b < p.n; b += kPiece)
            parts.push_back({p.o + b, static_cast<const char*>(p.src) + b, std::min(kPiece, p.n - b)});
        at = std::max(at, p.o + p.n);
    }
    if (P.plan_bytes > at) zero(at, P.plan_bytes - at);
    parallel_for((int64_t)parts.size(), [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) std::memcpy(dst + parts[i].o, parts[i].src, parts[i].n);
    }, parts.size() > 64 ? 8 : (int64_t)parts.size());
}

// The packed plan in host memory (for an upload from pageable memory).
struct PlanBlob {
    std::unique_ptr<char[]> p;
    size_t n = 0;
    const char* data() const { return p.get(); }
    size_t size() const { return n; }
};

static PlanBlob pack_plan(const Plan& P) {
    PlanBlob b;
    b.n = P.plan_bytes;
    b.p.reset(new char[std::max<size_t>(b.n, 1)]);
    pack_plan_into(P, b.p.get());
    return b;
}

// Chunks one decode wavefront takes unless a launch shape says otherwise.
static constexpr int kDefaultDecodeChunks = 8;

static int score_ctas() {
    static std::atomic<int> ctas{0};
    int c = ctas.load(std::memory_order_relaxed);
    if (c == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
        c = cus;  // one scoring work-group per compute unit (it holds ~150 KiB of LDS)
        ctas.store(c, std::memory_order_relaxed);
    }
    return c;
}


// Upload the plan, decode the batch's lists into tile buckets. Shared by top-K and dense.
// The plan bytes (pack_plan) are uploaded from src first unless src is null (already there).
static ebr_status run_decode(const Index& ix, const Plan& P, char* ws, hipStream_t st,
                             const char* src, size_t n_src, int chunks_per_wave) {
    if (src) HIP_TRY(hipMemcpyAsync(ws + P.off_plan, src, n_src, hipMemcpyHostToDevice, st));
    uint32_t* stcnt = (uint32_t*)(ws + P.off_stcnt);
    uint32_t* stoff = (uint32_t*)(ws + P.off_stoff);
    uint32_t* stfill = (uint32_t*)(ws + P.off_stfill);
    LAUNCH(launch_fill_u32(stcnt, 0u, P.n_super + 1, st));
    LAUNCH(launch_fill_u32(stfill, 0u, P.n_super + 1, st));
    DecodeArgs d{};
    d.chunks = ix.chunks;
    d.words = ix.words;
    d.weights = ix.weights;
    d.uk_chunk_begin = (const uint32_t*)(ws + P.o_ukb);
    d.uk_chunk_prefix = (const uint32_t*)(ws + P.o_ukp);
    d.uk_wshift = (const int32_t*)(ws + P.o_ukw);
    d.n_ukeys = P.nu;
    d.total_chunks = P.total_chunks;
    d.chunks_per_wave = (uint32_t)chunks_per_wave;
    d.n_tiles = ix.n_tiles;
    d.n_super = P.n_super;
    d.sshift = P.sshift;
    d.st_cnt = stcnt;
    d.st_off = stoff;
    d.st_fill = stfill;
    d.stage = (uint32_t*)(ws + P.off_stage);
    d.chunk_map = (uint2*)(ws + P.off_cmap);
    // one query group: bucket entries carry their key's users range directly
    d.users_off = P.packed ? (const uint32_t*)(ws + P.o_uoff) : nullptr;
    d.tile_off = (uint32_t*)(ws + P.off_toff);
    d.bucket = (uint32_t*)(ws + P.off_bucket);
    d.n_sub = P.n_sub;
    d.n_hot = P.n_hot;
    d.cold_first = P.split ? P.cold_first : P.nu;
    d.gq_shift = P.gq == 256 ? 8 : 7;
    d.cold_off = P.split ? (const uint32_t*)(ws + P.o_coff) : nullptr;
    d.cold_users = P.split ? (const uint32_t*)(ws + P.o_cusers) : nullptr;
    LAUNCH(launch_chunk_map(d, st));
    LAUNCH(launch_decode(d, 0, st));
    LAUNCH(launch_excl_scan_u32(stcnt, stoff, P.n_super, (uint32_t*)(ws + P.off_stmp), st));
    LAUNCH(launch_decode(d, 1, st));
    LAUNCH(launch_refine(d, st));
    return EBR_OK;
}

static ScoreArgs score_args(const Index& ix, const Plan& P, const ebr_batch* bt, char* ws) {
    ScoreArgs s{};
    s.dtype = P.dtype;
    s.emb = P.dtype == EBR_BF16 ? ix.emb_bf16 : (P.dtype == EBR_FP8E4M3 ? ix.emb_fp8 : ix.emb_f32);
    s.fp8_scale = ix.fp8_scale;
    s.n_ads = ix.n_ads;
    s.user = bt->user_emb;
    s.n_queries = P.B;
    s.n_qgroups = P.n_qg;
    s.packed = P.packed ? 1 : 0;
    s.wide64 = P.w64 ? 1 : 0;
    s.tile_off = (const uint32_t*)(ws + P.off_toff);
    s.bucket = (const uint32_t*)(ws + P.off_bucket);
    s.n_sub = P.n_sub;
    s.n_hot = P.n_hot;
    s.hot_tab = P.split ? (const uint32_t*)(ws + P.o_htab) : nullptr;
    s.hot_users = P.split ? (const uint32_t*)(ws + P.o_husers) : nullptr;
    s.hot_users_off = P.split ? (const uint32_t*)(ws + P.o_hoff) : nullptr;
    s.users_off = (const uint32_t*)(ws + P.o_uoff);
    s.users = (const uint32_t*)(ws + P.o_users);
    s.n_users = (uint32_t)P.nnz;
    s.qinv = (const double*)(ws + P.o_qi);
    s.n_work = (int32_t)ix.n_tiles;
    s.tile_list = nullptr;
    return s;
}

static ebr_status check_users(const ebr_batch* bt, int B, int dim, hipStream_t st,
                              std::vector<float>* host = nullptr) {
    if (B == 0) return EBR_OK;
    std::vector<float> local;
    std::vector<float>& u = host ? *host : local;
    u.resize((size_t)B * dim);
    HIP_TRY(hipMemcpyAsync(u.data(), bt->user_emb, u.size() * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (size_t i = 0; i < u.size(); ++i)
        if (!std::isfinite(u[i])) { set_error("query %zu: non-finite user embedding", i / dim); return EBR_EINVAL; }
    return EBR_OK;
}

// Key of the launch-shape table for FP32 batches with 64-bit cross-term cells (the scan dtypes
// are 0..2).
constexpr int kShapeKeyWide64 = 3;

// Launch shape of a batch: the override, else the one recorded for (dtype, query groups),
// else zeros (the defaults).
static ebr_launch_shape shape_for(const Index& ix, int dtype, int nqg, const ebr_launch_shape* over) {
    if (over) return *over;
    std::lock_guard<std::mutex> lk(ix.shape_mu);
    auto it = ix.shapes.find({dtype, nqg});
    return it == ix.shapes.end() ? ebr_launch_shape{} : it->second;
}

// The shape's fields with the defaults filled in, for a batch of nqg query groups.
static ebr_launch_shape effective_shape(const Index& ix, const ebr_launch_shape& sh, int64_t n_sample,
                                        int nqg) {
    ebr_launch_shape e = sh;
    if (e.score_ranges <= 0) e.score_ranges = score_ranges((int)ix.n_tiles, nqg, score_ctas());
    if (e.sample_ranges <= 0) e.sample_ranges = score_ranges((int)std::max<int64_t>(1, n_sample), nqg, score_ctas());
    if (e.decode_chunks <= 0) e.decode_chunks = kDefaultDecodeChunks;
    return e;
}

}  // namespace ebr

// A captured batch sequence: the capture stream, the executable graph, pinned plan staging.
struct ebr_graph {
    int device = 0;
    hipStream_t cs = nullptr;
    hipGraphExec_t exec = nullptr;
    char* pinned = nullptr;
    size_t pinned_cap = 0;
    ebr_graph_info info{};
    std::mutex mu;
};

namespace ebr {

// Load a captured sequence into the handle's executable graph (in place when only
// parameters changed) and launch it on s. Consumes `graph`.
static ebr_status graph_launch(ebr_graph* g, hipGraph_t graph, hipStream_t s) {
    size_t n = 0;
    if (hipGraphGetNodes(graph, nullptr, &n) != hipSuccess) n = 0;
    bool loaded = false;
    if (g->exec && n == g->info.nodes) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult r = hipGraphExecUpdateError;
        if (hipGraphExecUpdate(g->exec, graph, &bad, &r) == hipSuccess && r == hipGraphExecUpdateSuccess) {
            loaded = true;
            g->info.updates++;
        } else {
            (void)hipGetLastError();  // the update's refusal is not an error of the call
        }
    }
    if (!loaded) {
        if (g->exec) {
            (void)hipGraphExecDestroy(g->exec);
            g->exec = nullptr;
        }
        hipError_t e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            g->exec = nullptr;
            (void)hipGraphDestroy(graph);
            set_error("hipGraphInstantiate failed: %s", hipGetErrorString(e));
            return EBR_EDEVICE;
        }
        g->info.instantiations++;
    }
    g->info.nodes = n;
    (void)hipGraphDestroy(graph);
    HIP_TRY(hipGraphLaunch(g->exec, s));
    g->info.calls++;
    return EBR_OK;
}

struct TopkOpts {
    ebr_graph* graph = nullptr;             // capture the device sequence into this handle
    const ebr_launch_shape* shape = nullptr; // replaces the recorded shape
    bool force_timing = false;              // record phase times whatever ebr_set_timing says
};

static ebr_status topk_impl(const Index& ix, const ebr_batch* batch, char* ws, size_t ws_bytes,
                            uint32_t* out_ids, float* out_scores, hipStream_t s, ebr_timings* tm,
                            const TopkOpts& opt = TopkOpts{}) {
    const auto t_host = std::chrono::steady_clock::now();
    Plan P;
    ebr_status st = plan_batch(ix, batch, true, &P);
    if (st) return st;
    if (!ws || ws_bytes < P.total) { set_error("workspace too small: need %zu bytes, got %zu", P.total, ws_bytes); return EBR_ENOMEM; }
    if ((uintptr_t)ws & 255) { set_error("workspace must be 256-byte aligned"); return EBR_EINVAL; }
    const int64_t n_out = P.out_off[P.B];
    if (n_out > 0 && (!out_ids || !out_scores)) { set_error("NULL output"); return EBR_EINVAL; }
    if (P.B == 0) return EBR_OK;
    // the selection path: every query whose candidates fit the LDS sort
    auto selection = [&]() -> ebr_status {
        const bool approx = P.dtype != EBR_F32;
        const int64_t ns = (int64_t)P.sample_tiles.size();
        const ebr_launch_shape sh =
            effective_shape(ix, shape_for(ix, P.w64 ? kShapeKeyWide64 : P.dtype, P.n_qg, opt.shape), ns, P.n_qg);
        if (sh.score_ranges < 1 || sh.sample_ranges < 1 || sh.decode_chunks < 1 || sh.decode_chunks > 64) {
            set_error("launch shape out of range");
            return EBR_EINVAL;
        }
        ebr_graph* g = opt.graph;
        hipStream_t ls = s;  // the stream the device sequence is enqueued (or captured) on
        PlanBlob blob;
        const char* src = nullptr;
        if (g) {
            if (g->pinned_cap < P.plan_bytes) {
                if (g->pinned) (void)hipHostFree(g->pinned);
                g->pinned = nullptr;
                g->pinned_cap = 0;
                const size_t cap = std::max<size_t>(P.plan_bytes + P.plan_bytes / 4, 1 << 20);
                HIP_TRY(hipHostMalloc((void**)&g->pinned, cap, hipHostMallocDefault));
                g->pinned_cap = cap;
            }
            // packed straight into the pinned buffer; the plan goes up on the caller's stream
            // ahead of the graph, which holds kernels only
            pack_plan_into(P, g->pinned);
            HIP_TRY(hipMemcpyAsync(ws + P.off_plan, g->pinned, P.plan_bytes, hipMemcpyHostToDevice, s));
            ls = g->cs;
        } else {
            blob = pack_plan(P);
            src = blob.data();
        }
        const double host_ms = ms_since(t_host);
        PhaseClock clk(ls, !g && (opt.force_timing || g_timing.load() != 0));

        const int B = P.B;
        uint32_t* thr = (uint32_t*)(ws + P.off_thr);
        int32_t* status = (int32_t*)(ws + P.off_status);
        uint32_t* active = (uint32_t*)(ws + P.off_active);
        uint32_t* ccnt = (uint32_t*)(ws + P.off_ccnt);
        uint32_t* unres = (uint32_t*)(ws + P.off_unres);
        uint32_t* unc = (uint32_t*)(ws + P.off_unc);
        Control* ctl = (Control*)(ws + P.off_ctl);
        unsigned long long* cand = (unsigned long long*)(ws + P.off_cand);

        ScoreArgs sa = score_args(ix, P, batch, ws);
        sa.ctl = ctl;
        sa.n_work = (int32_t)ns;
        sa.tile_list = (const uint32_t*)(ws + P.o_st);
        sa.sample_keys = (uint32_t*)(ws + P.off_skeys);
        sa.sample_ld = ns * kTileAds;
        SelectArgs se{};
        se.keys = sa.sample_keys;
        se.ld = sa.sample_ld;
        se.n_cols = sa.sample_ld;
        se.jq = (const int32_t*)(ws + P.o_jq);
        se.kq = (const int32_t*)(ws + P.o_kq);
        se.kcnt = (const int32_t*)(ws + P.o_kc);
        se.n_valid = P.n_sample_valid;
        se.status = status;
        se.only_status = -1;
        // Test hook: EBR_FORCE_SELECT_ROUND = 1 or 2 makes the first threshold follow the rule of
        // that revision round (1: the sample's K'-th key; 2: no threshold, every ad a candidate),
        // so that the rounds' thresholds are exercised on ordinary inputs.
        if (const char* fr = std::getenv("EBR_FORCE_SELECT_ROUND")) {
            if (fr[0] == '1' && fr[1] == '\0') se.round = 1;
            if (fr[0] == '2' && fr[1] == '\0') se.round = 2;
        }
        se.thresh = thr;
        se.ctl = ctl;
        ScoreArgs ca = score_args(ix, P, batch, ws);
        ca.ctl = ctl;
        ca.thresh = thr;
        ca.active = active;
        ca.cand = cand;
        ca.cand_wide = approx ? (float*)(ws + P.off_cwide) : nullptr;
        ca.cand_cnt = ccnt;
        ca.cap = kCandCap;
        FinalArgs fa{};
        fa.ctl = ctl;
        fa.active = active;
        fa.kq = (const int32_t*)(ws + P.o_kq);
        fa.kcnt = (const int32_t*)(ws + P.o_kc);
        fa.cand_cnt = ccnt;
        fa.cap = kCandCap;
        fa.cand = cand;
        fa.cand_wide = ca.cand_wide;
        fa.status = status;
        fa.thresh = thr;
        fa.prep = approx ? 1 : 0;
        fa.out_off = (const int64_t*)(ws + P.o_oo);
        fa.out_ids = out_ids;
        fa.out_scores = out_scores;
        fa.werr = P.w64 ? nullptr : (const float*)(ws + P.o_werr);
        fa.imprecise = &ctl->imprecise;
        if (approx) {
            fa.r_id = (uint32_t*)(ws + P.off_rid);
            fa.r_wide = (float*)(ws + P.off_rwide);
            fa.r_stilde = (float*)(ws + P.off_rst);
            fa.r_ld = std::max(1, P.kcmax);
        }
        RescoreArgs ra{};
        ra.ctl = ctl;
        ra.emb = ix.emb_f32;
        ra.user = batch->user_emb;
        ra.n_ads = ix.n_ads;
        ra.kq = fa.kq;
        ra.kcnt = fa.kcnt;
        ra.status = status;
        ra.uncertified = unc;
        ra.r_id = fa.r_id;
        ra.r_wide = fa.r_wide;
        ra.r_stilde = fa.r_stilde;
        ra.eps = (const float*)(ws + P.off_eps);
        ra.werr = fa.werr;
        ra.imprecise = fa.imprecise;
        ra.r_ld = fa.r_ld;
        ra.out_off = fa.out_off;
        ra.out_ids = out_ids;
        ra.out_scores = out_scores;

        int e_dec0 = -1, e_dec1 = -1, e_smp1 = -1, e_rs0 = -1, e_rs1 = -1;
        std::vector<std::array<int, 3>> round_marks;
        // The device sequence of the batch, enqueued on ls without host synchronisation.
        auto enqueue = [&]() -> ebr_status {
            e_dec0 = clk.mark();
            ebr_status r = run_decode(ix, P, ws, ls, src, P.plan_bytes, sh.decode_chunks);
            if (r) return r;
            e_dec1 = clk.mark();
            // per-query set-up on the device: user rows finite, status / activity, certificate eps
            LAUNCH(launch_fill_u32((uint32_t*)ctl, 0u, (int64_t)(sizeof(Control) / 4), ls));
            PrepArgs pa{};
            pa.user = batch->user_emb;
            pa.n_queries = B;
            pa.dim = ix.dim;
            pa.kq = (const int32_t*)(ws + P.o_kq);
            pa.aq = (const double*)(ws + P.o_aq);
            pa.status = status;
            pa.active = active;
            pa.eps = approx ? (float*)(ws + P.off_eps) : nullptr;
            const int cq = P.dtype == EBR_BF16 ? 0 : 1;
            pa.q_err2 = ix.q_err2[cq];
            pa.q_norm2 = ix.q_norm2[cq];
            pa.e_norm2 = ix.e_norm2;
            pa.ctl = ctl;
            LAUNCH(launch_prep(pa, ls));
            // sample pass and per-query threshold (for K' candidates on approximate scans)
            LAUNCH(launch_score(sa, ix.dim, 1, sh.sample_ranges, ls));
            LAUNCH(launch_select(se, B, ls));
            se.round = 0;
            e_smp1 = clk.mark();
            // Selection rounds: round r > 0 runs only if round r - 1 left a query unresolved.
            // Queries short of K' candidates first take the sample's K'-th key (which at least
            // K' sample ads reach), then no threshold at all; overflowing queries take the
            // K'-th largest stored key.
            for (int rr = 0; rr < kMaxRounds; ++rr) {
                const uint32_t* gate = rr == 0 ? nullptr : &ctl->unres[rr - 1];
                if (rr > 0) {
                    se.gate = gate;
                    se.round = rr;
                    se.only_status = kStatusNeedLower;
                    LAUNCH(launch_select(se, B, ls));
                }
                LAUNCH(launch_round_reset(ccnt, B, gate, ls));
                ca.gate = gate;
                fa.gate = gate;
                fa.unresolved = &ctl->unres[rr];
                const int e0 = clk.mark();
                LAUNCH(launch_score(ca, ix.dim, 0, sh.score_ranges, ls));
                const int e1 = clk.mark();
                LAUNCH(launch_finalize(fa, B, ls));
                const int e2 = clk.mark();
                round_marks.push_back({e0, e1, e2});
            }
            if (approx) {
                // exact FP32 rescore of the K' candidates, top K, recall certificate; skipped
                // while a query is still unresolved (then it runs after the extra rounds)
                LAUNCH(launch_fill_u32(unc, 0u, 1, ls));
                ra.skip = &ctl->unres[kMaxRounds - 1];
                e_rs0 = clk.mark();
                LAUNCH(launch_rescore(ra, ix.dim, B, ls));
                e_rs1 = clk.mark();
            }
            return EBR_OK;
        };

        if (g) {
            HIP_TRY(hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal));
            const ebr_status r = enqueue();
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(ls, &graph);
            if (r || ec != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                if (!r) set_error("hipStreamEndCapture failed: %s", hipGetErrorString(ec));
                return r ? r : EBR_EDEVICE;
            }
            st = graph_launch(g, graph, s);
            if (st) return st;
        } else {
            st = enqueue();
            if (st) return st;
        }

        Control hc{};
        uint32_t nunc = 0;
        HIP_TRY(hipMemcpyAsync(&hc, ctl, sizeof(Control), hipMemcpyDeviceToHost, s));
        if (approx) HIP_TRY(hipMemcpyAsync(&nunc, unc, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hc.error & 1u) { set_error("non-finite user embedding in the batch"); return EBR_EINVAL; }
        if (hc.error & 4u) { set_error("internal error: a rescore candidate id lies outside the inventory"); return EBR_EDEVICE; }
        int rounds_run = 1;
        for (int r = 0; r + 1 < kMaxRounds; ++r) rounds_run += hc.unres[r] > 0 ? 1 : 0;
        // rare: still unresolved after the enqueued rounds; continue round by round
        const bool extra = hc.unres[kMaxRounds - 1] > 0;
        for (int r = kMaxRounds; hc.unres[kMaxRounds - 1] > 0; ++r) {
            if (r >= 64) { set_error("top-K selection did not converge"); return EBR_EDEVICE; }
            se.gate = nullptr;
            se.round = 2;
            se.only_status = kStatusNeedLower;
            LAUNCH(launch_select(se, B, s));
            LAUNCH(launch_round_reset(ccnt, B, nullptr, s));
            ca.gate = nullptr;
            fa.gate = nullptr;
            LAUNCH(launch_fill_u32(unres, 0u, 1, s));
            fa.unresolved = unres;
            LAUNCH(launch_score(ca, ix.dim, 0, sh.score_ranges, s));
            LAUNCH(launch_finalize(fa, B, s));
            uint32_t left = 0;
            HIP_TRY(hipMemcpyAsync(&left, unres, 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            ++rounds_run;
            hc.unres[kMaxRounds - 1] = left;
        }
        if (approx && extra) {
            ra.skip = nullptr;
            LAUNCH(launch_fill_u32(unc, 0u, 1, s));
            LAUNCH(launch_rescore(ra, ix.dim, B, s));
            HIP_TRY(hipMemcpyAsync(&nunc, unc, 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        // cross-term precision checks of the finalize / rescore kernels run after the rounds
        uint32_t nimp = hc.imprecise;
        if (extra) {
            HIP_TRY(hipMemcpyAsync(&nimp, &ctl->imprecise, 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        const int n_unc = (int)nunc, n_imp = (int)nimp;
        if (tm) {
            tm->host_ms = host_ms;
            tm->decode_ms = clk.ms(e_dec0, e_dec1);
            tm->sample_ms = clk.ms(e_dec1, e_smp1);
            for (const auto& r : round_marks) {
                tm->score_ms += clk.ms(r[0], r[1]);
                tm->finalize_ms += clk.ms(r[1], r[2]);
            }
            tm->score_first_ms = round_marks.empty() ? 0.0 : clk.ms(round_marks[0][0], round_marks[0][1]);
            tm->rescore_ms = clk.ms(e_rs0, e_rs1);
            tm->rounds = rounds_run;
            tm->uncertified = n_unc;
            tm->imprecise = n_imp;
        }
        if (n_unc > 0 || n_imp > 0) {
            // rare: queries whose recall certificate failed run again on the FP32 scan, queries
            // whose 32-bit cross term was too coarse with 64-bit cells; each subset as a batch of
            // its own in the bytes below fb_limit, results copied into place
            std::vector<int32_t> sv(B);
            HIP_TRY(hipMemcpyAsync(sv.data(), status, 4 * (size_t)B, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            float* fu = (float*)(ws + P.off_fb_users);
            uint32_t* fids = (uint32_t*)(ws + P.off_fb_ids);
            float* fsc = (float*)(ws + P.off_fb_scores);
            auto rerun = [&](int want, bool w64) -> ebr_status {
                std::vector<int> fq;
                for (int q = 0; q < B; ++q)
                    if (sv[q] == want) fq.push_back(q);
                const int nb = (int)fq.size();
                if (nb == 0) return EBR_OK;
                std::vector<int64_t> foff(nb + 1, 0);
                std::vector<int32_t> fkeys, fk(nb);
                std::vector<float> fmult;
                for (int i = 0; i < nb; ++i) {
                    const int q = fq[i];
                    HIP_TRY(hipMemcpyAsync(fu + (size_t)i * ix.dim, batch->user_emb + (size_t)q * ix.dim,
                                           4 * (size_t)ix.dim, hipMemcpyDeviceToDevice, s));
                    for (int64_t j = batch->feat_offsets[q]; j < batch->feat_offsets[q + 1]; ++j) {
                        fkeys.push_back(batch->feat_keys[j]);
                        if (batch->feat_mult) fmult.push_back(batch->feat_mult[j]);
                    }
                    foff[i + 1] = (int64_t)fkeys.size();
                    fk[i] = P.kq[q];
                }
                ebr_batch fb{};
                fb.n_queries = nb;
                fb.user_emb = fu;
                fb.feat_offsets = foff.data();
                fb.feat_keys = fkeys.data();
                fb.feat_mult = batch->feat_mult ? fmult.data() : nullptr;
                fb.k = fk.data();
                fb.scan_dtype = EBR_F32;
                fb.rescore_factor = 0;
                fb.wide64 = w64 ? 1 : 0;
                ebr_status r = topk_impl(ix, &fb, ws, P.fb_limit, fids, fsc, s, nullptr);
                if (r) return r;
                int64_t pos = 0;
                for (int i = 0; i < nb; ++i) {
                    const int q = fq[i];
                    const size_t n = (size_t)P.kq[q];
                    HIP_TRY(hipMemcpyAsync(out_ids + P.out_off[q], fids + pos, 4 * n, hipMemcpyDeviceToDevice, s));
                    HIP_TRY(hipMemcpyAsync(out_scores + P.out_off[q], fsc + pos, 4 * n, hipMemcpyDeviceToDevice, s));
                    pos += (int64_t)n;
                }
                HIP_TRY(hipStreamSynchronize(s));
                return EBR_OK;
            };
            st = rerun(kStatusUncertified, false);
            if (st) return st;
            st = rerun(kStatusImprecise, true);
            if (st) return st;
        }
        return EBR_OK;
    };
    if (P.kmax > 0) {
        st = selection();
        if (st) return st;
    }
    // queries whose K (or K' = factor x K) exceeds the LDS sort: one full sort each, on the
    // FP32 scan with 64-bit cross-term cells, written at the query's offsets
    for (const int q : P.big) {
        ebr_batch b1{};
        const int64_t f0 = batch->feat_offsets[q];
        const int64_t foff[2] = {0, batch->feat_offsets[q + 1] - f0};
        b1.n_queries = 1;
        b1.user_emb = batch->user_emb + (size_t)q * ix.dim;
        b1.feat_offsets = foff;
        b1.feat_keys = batch->feat_keys ? batch->feat_keys + f0 : nullptr;
        b1.feat_mult = batch->feat_mult ? batch->feat_mult + f0 : nullptr;
        b1.scan_dtype = EBR_F32;
        b1.wide64 = 1;
        st = check_users(&b1, 1, ix.dim, s);
        if (st) return st;
        Plan Pd;
        st = plan_batch(ix, &b1, false, &Pd);
        if (st) return st;
        if (Pd.total > P.off_big_deep) { set_error("full-sort plan exceeds its workspace"); return EBR_EDEVICE; }
        const PlanBlob blob = pack_plan(Pd);
        st = run_decode(ix, Pd, ws, s, blob.data(), blob.size(), kDefaultDecodeChunks);
        if (st) return st;
        float* deep = (float*)(ws + P.off_big_deep);
        float* wide = (float*)(ws + P.off_big_wide);
        ScoreArgs a = score_args(ix, Pd, &b1, ws);
        a.deep_out = deep;
        a.wide_out = wide;
        LAUNCH(launch_score(a, ix.dim, 2, score_ranges((int)ix.n_tiles, Pd.n_qg, score_ctas()), s));
        const int64_t o = P.out_off[q], k = P.out_off[q + 1] - o;
        LAUNCH(launch_full_sort_topk(deep, wide, ix.n_ads, k, (unsigned long long*)(ws + P.off_big_keys),
                                     (unsigned long long*)(ws + P.off_big_tmp), (uint32_t*)(ws + P.off_big_hist),
                                     (uint32_t*)(ws + P.off_big_stmp), out_ids + o, out_scores + o, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return EBR_OK;
}

ebr_status run_topk(const Index& ix, const ebr_batch* batch, char* ws, size_t ws_bytes,
                    uint32_t* out_ids, float* out_scores, void* stream, ebr_timings* tm,
                    ebr_graph* graph, const ebr_launch_shape* shape) {
    TopkOpts o;
    o.graph = graph;
    o.shape = shape;
    if (!graph) return topk_impl(ix, batch, ws, ws_bytes, out_ids, out_scores, (hipStream_t)stream, tm, o);
    std::lock_guard<std::mutex> lk(graph->mu);
    return topk_impl(ix, batch, ws, ws_bytes, out_ids, out_scores, (hipStream_t)stream, tm, o);
}

size_t topk_workspace_bytes(const Index& ix, int dtype, BatchSizes z) {
    z.n_sample = z.n_out > 0 ? sample_tile_count(ix, z.kcmax) : 0;
    return layout_total(ix, z, dtype, false);
}

}  // namespace ebr

extern "C" {

ebr_status ebr_workspace_size(const ebr_index* index, const ebr_batch* batch, size_t* bytes) {
    try {
        if (!index || !bytes) { set_error("NULL argument"); return EBR_EINVAL; }
        Plan P;
        ebr_status st = plan_batch(*index, batch, true, &P);
        if (st) return st;
        *bytes = P.total;
        return EBR_OK;
    } catch (const std::bad_alloc&) {
        set_error("host out of memory");
        return EBR_ENOMEM;
    }
}

ebr_status ebr_score_topk(const ebr_index* index, const ebr_batch* batch, void* ws_v,
                          size_t ws_bytes, uint32_t* out_ids, float* out_scores, void* hip_stream) {
    try {
        if (!index) { set_error("index is NULL"); return EBR_EINVAL; }
        g_last_timings = ebr_timings{};
        return topk_impl(*index, batch, (char*)ws_v, ws_bytes, out_ids, out_scores,
                         (hipStream_t)hip_stream, &g_last_timings);
    } catch (const std::bad_alloc&) {
        set_error("host out of memory");
        return EBR_ENOMEM;
    }
}

static bool shape_ok(const ebr_launch_shape& sh) {
    return sh.score_ranges >= 0 && sh.score_ranges <= (1 << 24) && sh.sample_ranges >= 0 &&
           sh.sample_ranges <= (1 << 24) && sh.decode_chunks >= 0 && sh.decode_chunks <= 64;
}

static int query_groups(const ebr_index* index, int32_t n_queries) {
    const int gq = score_group_queries(index->dim);
    return (int)(((int64_t)n_queries + gq - 1) / gq);
}

ebr_status ebr_set_launch_shape(ebr_index* index, ebr_dtype scan_dtype, int32_t n_queries,
                                const ebr_launch_shape* shape) {
    if (!index) { set_error("index is NULL"); return EBR_EINVAL; }
    if (n_queries < 1 || scan_dtype < EBR_F32 || scan_dtype > EBR_FP8E4M3) { set_error("bad dtype or query count"); return EBR_EINVAL; }
    if (shape && !shape_ok(*shape)) { set_error("launch shape out of range"); return EBR_EINVAL; }
    try {
        std::lock_guard<std::mutex> lk(index->shape_mu);
        const std::pair<int, int> key{(int)scan_dtype, query_groups(index, n_queries)};
        if (shape) index->shapes[key] = *shape;
        else index->shapes.erase(key);
    } catch (const std::bad_alloc&) {
        set_error("host out of memory");
        return EBR_ENOMEM;
    }
    return EBR_OK;
}

ebr_status ebr_get_launch_shape(const ebr_index* index, ebr_dtype scan_dtype, int32_t n_queries,
                                ebr_launch_shape* out) {
    if (!index || !out) { set_error("NULL argument"); return EBR_EINVAL; }
    if (n_queries < 1 || scan_dtype < EBR_F32 || scan_dtype > EBR_FP8E4M3) { set_error("bad dtype or query count"); return EBR_EINVAL; }
    *out = shape_for(*index, (int)scan_dtype, query_groups(index, n_queries), nullptr);
    return EBR_OK;
}

ebr_status ebr_autotune(ebr_index* index, const ebr_batch* batch, void* ws_v, size_t ws_bytes,
                        uint32_t* out_ids, float* out_scores, int32_t reps, void* hip_stream,
                        ebr_tune_report* out) {
    try {
        if (!index) { set_error("index is NULL"); return EBR_EINVAL; }
        const Index& ix = *index;
        ebr_tune_report rep{};
        if (out) *out = rep;
        Plan P;
        ebr_status st = plan_batch(ix, batch, true, &P);
        if (st) return st;
        hipStream_t s = (hipStream_t)hip_stream;
        char* ws = (char*)ws_v;
        TopkOpts o;
        o.force_timing = true;
        if (P.B == 0 || P.kmax == 0)  // nothing runs on the device: nothing to tune
            return topk_impl(ix, batch, ws, ws_bytes, out_ids, out_scores, s, nullptr, o);
        reps = reps <= 0 ? 3 : std::min(reps, 64);
        const int nqg = P.n_qg;
        const int64_t ns = (int64_t)P.sample_tiles.size();
        // device time of the batch under a shape: the median over reps of the summed phases
        auto run = [&](const ebr_launch_shape& sh, float* ms) -> ebr_status {
            std::vector<double> t;
            o.shape = &sh;
            for (int r = 0; r < reps; ++r) {
                ebr_timings tm{};
                ebr_status e = topk_impl(ix, batch, ws, ws_bytes, out_ids, out_scores, s, &tm, o);
                if (e) return e;
                t.push_back(tm.decode_ms + tm.sample_ms + tm.score_ms + tm.finalize_ms + tm.rescore_ms);
            }
            std::sort(t.begin(), t.end());
            *ms = (float)t[t.size() / 2];
            return EBR_OK;
        };
        ebr_launch_shape best = effective_shape(ix, ebr_launch_shape{}, ns, nqg);
        {
            ebr_timings tm{};
            o.shape = &best;
            st = topk_impl(ix, batch, ws, ws_bytes, out_ids, out_scores, s, &tm, o);  // untimed
            if (st) return st;
        }
        float best_ms = 0.0f;
        st = run(best, &best_ms);
        if (st) return st;
        rep.tried[0] = best;
        rep.tried_ms[0] = best_ms;
        rep.default_ms = best_ms;
        rep.n_tried = 1;
        auto consider = [&](ebr_launch_shape c) -> ebr_status {
            c = effective_shape(ix, c, ns, nqg);
            if (c.score_ranges == best.score_ranges && c.sample_ranges == best.sample_ranges &&
                c.decode_chunks == best.decode_chunks)
                return EBR_OK;
            if (rep.n_tried >= EBR_TUNE_MAX) return EBR_OK;
            float ms = 0.0f;
            const ebr_status e = run(c, &ms);
            if (e) return e;
            rep.tried[rep.n_tried] = c;
            rep.tried_ms[rep.n_tried] = ms;
            rep.n_tried++;
            if (ms < 0.99f * best_ms) {  // 1% margin: ties keep the earlier shape
                best = c;
                best_ms = ms;
            }
            return EBR_OK;
        };
        const int cus = score_ctas();
        auto ranges_at = [&](int per_cu, int64_t n_work) {
            int R = (int)std::max<int64_t>(1, (int64_t)per_cu * cus / nqg);
            if (R >= 8) R -= R % 8;
            return (int)std::min<int64_t>(R, std::max<int64_t>(1, n_work));
        };
        for (int m : {1, 2, 4}) {
            ebr_launch_shape c = best;
            c.score_ranges = ranges_at(m, ix.n_tiles);
            st = consider(c);
            if (st) return st;
        }
        for (int m : {1, 2, 4}) {
            ebr_launch_shape c = best;
            c.sample_ranges = ranges_at(m, ns);
            st = consider(c);
            if (st) return st;
        }
        for (int dc : {4, 8, 16, 32}) {
            ebr_launch_shape c = best;
            c.decode_chunks = dc;
            st = consider(c);
            if (st) return st;
        }
        rep.best = best;
        rep.best_ms = best_ms;
        {
            std::lock_guard<std::mutex> lk(index->shape_mu);
            index->shapes[{P.w64 ? kShapeKeyWide64 : P.dtype, nqg}] = best;
        }
        // leave the winner's results in the outputs
        o.shape = &best;
        st = topk_impl(ix, batch, ws, ws_bytes, out_ids, out_scores, s, nullptr, o);
        if (st) return st;
        if (out) *out = rep;
        return EBR_OK;
    } catch (const std::bad_alloc&) {
        set_error("host out of memory");
        return EBR_ENOMEM;
    }
}

ebr_status ebr_graph_create(ebr_graph** out) {
    if (!out) { set_error("NULL argument"); return EBR_EINVAL; }
    *out = nullptr;
    ebr_graph* g = new (std::nothrow) ebr_graph();
    if (!g) { set_error("host out of memory"); return EBR_ENOMEM; }
    hipError_t e = hipGetDevice(&g->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&g->cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete g;
        set_error("graph stream: %s", hipGetErrorString(e));
        return EBR_EDEVICE;
    }
    *out = g;
    return EBR_OK;
}

ebr_status ebr_score_topk_graph(ebr_graph* graph, const ebr_index* index, const ebr_batch* batch,
                                void* ws_v, size_t ws_bytes, uint32_t* out_ids, float* out_scores,
                                void* hip_stream) {
    try {
        if (!graph || !index) { set_error("NULL handle"); return EBR_EINVAL; }
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess || dev != graph->device) {
            set_error("graph handle belongs to device %d", graph->device);
            return EBR_EINVAL;
        }
        TopkOpts o;
        o.graph = graph;
        // the handle's staging, stream and executable graph serve one call at a time
        std::lock_guard<std::mutex> lk(graph->mu);
        return topk_impl(*index, batch, (char*)ws_v, ws_bytes, out_ids, out_scores,
                         (hipStream_t)hip_stream, nullptr, o);
    } catch (const std::bad_alloc&) {
        set_error("host out of memory");
        return EBR_ENOMEM;
    }
}

ebr_status ebr_graph_stats(const ebr_graph* graph, ebr_graph_info* out) {
    if (!graph || !out) { set_error("NULL argument"); return EBR_EINVAL; }
    *out = graph->info;
    return EBR_OK;
}

void ebr_graph_destroy(ebr_graph* graph) {
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->cs) (void)hipStreamDestroy(graph->cs);
    if (graph->pinned) (void)hipHostFree(graph->pinned);
    delete graph;
}

ebr_status ebr_score_dense(const ebr_index* index, const ebr_batch* batch, void* ws_v,
                           size_t ws_bytes, float* deep, float* wide, void* hip_stream) {
    try {
        if (!index) { set_error("index is NULL"); return EBR_EINVAL; }
        const Index& ix = *index;
        Plan P;
        ebr_status st = plan_batch(ix, batch, false, &P);
        if (st) return st;
        if (!ws_v || ws_bytes < P.total) { set_error("workspace too small: need %zu bytes, got %zu", P.total, ws_bytes); return EBR_ENOMEM; }
        if ((uintptr_t)ws_v & 255) { set_error("workspace must be 256-byte aligned"); return EBR_EINVAL; }
        if (P.B == 0) return EBR_OK;
        if (!deep || !wide) { set_error("NULL output"); return EBR_EINVAL; }
        hipStream_t s = (hipStream_t)hip_stream;
        st = check_users(batch, P.B, ix.dim, s);
        if (st) return st;
        char* ws = (char*)ws_v;
        const PlanBlob blob = pack_plan(P);
        st = run_decode(ix, P, ws, s, blob.data(), blob.size(), kDefaultDecodeChunks);
        if (st) return st;
        ScoreArgs a = score_args(ix, P, batch, ws);
        a.deep_out = deep;
        a.wide_out = wide;
        LAUNCH(launch_score(a, ix.dim, 2, score_ranges((int)ix.n_tiles, P.n_qg, score_ctas()), s));
        HIP_TRY(hipStreamSynchronize(s));
        return EBR_OK;
    } catch (const std::bad_alloc&) {
        set_error("host out of memory");
        return EBR_ENOMEM;
    }
}

// ---------------------------------------------------------------- codec (host)

ebr_status ebr_codec_size(const uint32_t* ids, int64_t n, size_t* bytes) {
    if (!bytes || n < 0 || (n > 0 && !ids)) { set_error("bad argument"); return EBR_EINVAL; }
    for (int64_t i = 1; i < n; ++i)
        if (ids[i] <= ids[i - 1]) { set_error("ids not strictly increasing at %lld", (long long)i); return EBR_EINVAL; }
    int64_t c, w;
    codec_measure(ids, n, &c, &w);
    *bytes = (size_t)c * 16 + (size_t)w * 4;
    return EBR_OK;
}

ebr_status ebr_codec_encode(const uint32_t* ids, int64_t n, void* out, size_t cap, size_t* used) {
    size_t need;
    ebr_status st = ebr_codec_size(ids, n, &need);
    if (st) return st;
    if (!out || cap < need) { set_error("output too small: need %zu", need); return EBR_ENOMEM; }
    int64_t c, w;
    codec_measure(ids, n, &c, &w);
    std::vector<ChunkHdr> hdr((size_t)c);
    std::vector<uint32_t> words((size_t)w + 1, 0u);
    codec_encode(ids, n, hdr.data(), words.data(), 0, 0);
    std::memcpy(out, hdr.data(), (size_t)c * 16);
    std::memcpy((char*)out + (size_t)c * 16, words.data(), (size_t)w * 4);
    if (used) *used = need;
    return EBR_OK;
}

ebr_status ebr_codec_decode(const void* in, size_t bytes, int64_t n, uint32_t* ids) {
    if (n < 0 || (n > 0 && (!in || !ids))) { set_error("bad argument"); return EBR_EINVAL; }
    const int64_t c = (n + kChunk - 1) / kChunk;
    if (bytes < (size_t)c * 16 || (bytes - (size_t)c * 16) % 4) { set_error("malformed encoding size"); return EBR_EINVAL; }
    std::vector<ChunkHdr> hdr((size_t)c);
    std::memcpy(hdr.data(), in, (size_t)c * 16);
    const int64_t nw = (int64_t)((bytes - (size_t)c * 16) / 4);
    std::vector<uint32_t> words((size_t)nw + 1, 0u);
    std::memcpy(words.data(), (const char*)in + (size_t)c * 16, (size_t)nw * 4);
    if (!codec_decode(hdr.data(), c, words.data(), nw, n, ids)) { set_error("malformed encoding"); return EBR_EINVAL; }
    return EBR_OK;
}

}  // extern "C"
