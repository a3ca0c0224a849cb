// gfx950 (CDNA4) kernels of libebr.
//
// One batch of queries runs as:
//   1. k_decode (count)  - every chunk of every distinct key of the batch is decoded by one
//                          wavefront; postings are counted per 32-ad tile.
//   2. scan              - exclusive scan of the tile counts.
//   3. k_decode (place)  - decode again and place each posting (key slot, ad, weight) into
//                          its tile's bucket: the batch's postings, tile-major.
//   4. k_score (sample)  - full scores of an evenly spread sample of tiles.
//   5. k_select          - per query, a radix select over the sample gives a score
//                          threshold that at least j sample ads reach.
//   6. k_score (collect) - every tile: cross term accumulated in LDS from the tile's bucket,
//                          dot products on the matrix cores, survivors of the threshold
//                          appended to per-query candidate buffers.
//   7. k_finalize        - per query, a bitonic sort of the candidates in LDS and the first
//                          K written out; queries whose candidate count fell outside
//                          [K, capacity] get a tighter or safer threshold and run again.
//
// The cross term of Section 3.3 (equation "hitmatch") is accumulated as 64-bit fixed point.
// Each posting weight of key k is rounded to w_fix = round(w * 2^Sw_k) (|w_fix| < 2^30) when
// it is placed into its bucket; each (query, key) multiplier to m_fix = round(m * 2^(S_q -
// Sw_k)) on the host, so m_fix * w_fix ~ m * w * 2^S_q at one common per-query scale with
// sum |m_fix * w_fix| < 2^60. Integer sums do not depend on the order in which postings are
// added, so scores are bit-identical across passes, tile schedules and batch compositions.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "kernels.h"

namespace ebr {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------------ small helpers

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Orderable key of an FP32 score: larger score <=> larger key; -0.0 maps like +0.0.
__device__ __forceinline__ uint32_t score_key(float s) {
    uint32_t u = __float_as_uint(s + 0.0f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_score(uint32_t k) {
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

// Block-wide exclusive scan for blockDim.x == NT (multiple of 64). sbuf holds NT/64 + 1 words.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sbuf, uint32_t* total) {
    constexpr int NW = NT / 64;
    const int lane = lane_id(), wave = (int)(threadIdx.x >> 6);
    uint32_t incl = wave_incl_scan(v);
    if (lane == 63) sbuf[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < NW; ++w) {
            uint32_t t = sbuf[w];
            sbuf[w] = run;
            run += t;
        }
        sbuf[NW] = run;
    }
    __syncthreads();
    uint32_t r = incl - v + sbuf[wave];
    *total = sbuf[NW];
    __syncthreads();
    return r;
}

// ------------------------------------------------------------------ fill / scan

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

constexpr int kScanNT = 256, kScanPer = 16, kScanBlock = kScanNT * kScanPer;

__global__ __launch_bounds__(kScanNT) void k_scan_reduce(const uint32_t* in, int64_t n,
                                                         uint32_t* partial) {
    __shared__ uint32_t red[kScanNT / 64];
    int64_t base = (int64_t)blockIdx.x * kScanBlock;
    uint32_t s = 0;
    for (int i = 0; i < kScanPer; ++i) {
        int64_t idx = base + (int64_t)i * kScanNT + threadIdx.x;
        if (idx < n) s += in[idx];
    }
    s = wave_incl_scan(s);
    if (lane_id() == 63) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kScanNT / 64; ++w) t += red[w];
        partial[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t* partial, int64_t np) {
    __shared__ uint32_t sbuf[1024 / 64 + 1];
    uint32_t carry = 0;
    for (int64_t base = 0; base < np; base += 1024) {
        int64_t i = base + threadIdx.x;
        uint32_t v = i < np ? partial[i] : 0;
        uint32_t tot;
        uint32_t e = block_excl_scan<1024>(v, sbuf, &tot);
        if (i < np) partial[i] = e + carry;
        carry += tot;
    }
}

__global__ __launch_bounds__(kScanNT) void k_scan_apply(const uint32_t* in, int64_t n,
                                                        const uint32_t* partial, uint32_t* out) {
    __shared__ uint32_t sbuf[kScanNT / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * kScanBlock;
    uint32_t carry = partial[blockIdx.x];
    for (int i = 0; i < kScanPer; ++i) {
        int64_t idx = base + (int64_t)i * kScanNT + threadIdx.x;
        uint32_t v = idx < n ? in[idx] : 0;
        uint32_t tot;
        uint32_t e = block_excl_scan<kScanNT>(v, sbuf, &tot);
        if (idx < n) out[idx] = e + carry;
        if (idx == n) out[n] = e + carry;
        carry += tot;
    }
}

// ------------------------------------------------------------------ chunk decode

// Decode chunk `chunk`: returns this lane's id (lanes >= count return garbage, valid=false).
__device__ __forceinline__ uint32_t decode_chunk_lane(const ChunkHdr* chunks, const uint32_t* words,
                                                      uint32_t chunk, int* count_out,
                                                      uint32_t* post_off_out) {
    const int lane = lane_id();
    const uint4 h = *reinterpret_cast<const uint4*>(chunks + chunk);
    const int b = (int)(h.y & 63u);
    const int count = (int)((h.y >> 8) & 127u);
    uint32_t gap = 0;
    if (lane >= 1 && lane < count && b > 0) {
        uint32_t bitpos = (uint32_t)(lane - 1) * (uint32_t)b;
        const uint32_t* w = words + h.z + (bitpos >> 5);
        uint64_t v = ((uint64_t)w[1] << 32) | (uint64_t)w[0];
        v >>= (bitpos & 31u);
        gap = (b == 32) ? (uint32_t)v : ((uint32_t)v & ((1u << b) - 1u));
    }
    uint32_t delta = (lane >= 1 && lane < count) ? gap + 1u : 0u;
    uint32_t id = h.x + wave_incl_scan(delta);
    *count_out = count;
    *post_off_out = h.w;
    return id;
}

constexpr int kChunksPerWave = 8;

// One wavefront decodes kChunksPerWave consecutive chunks of the batch's distinct keys and
// counts (place == 0) or places (place == 1) their postings into 32-ad tile buckets. Runs
// of postings in the same tile are aggregated into one atomic per run.
__global__ __launch_bounds__(256) void k_decode(DecodeArgs a, int place) {
    const int lane = lane_id();
    const uint32_t gw = blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t c_begin = gw * (uint32_t)kChunksPerWave;
    if (c_begin >= a.total_chunks) return;
    const uint32_t c_end = min(a.total_chunks, c_begin + (uint32_t)kChunksPerWave);
    // distinct-key slot owning the first chunk: the last u with prefix[u] <= c_begin
    int lo = 0, hi = a.n_ukeys;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (a.uk_chunk_prefix[mid] <= c_begin) lo = mid; else hi = mid;
    }
    uint32_t u = (uint32_t)lo;
    for (uint32_t gc = c_begin; gc < c_end; ++gc) {
        while (a.uk_chunk_prefix[u + 1] <= gc) ++u;
        const uint32_t chunk = a.uk_chunk_begin[u] + (gc - a.uk_chunk_prefix[u]);
        int count;
        uint32_t post_off;
        const uint32_t id = decode_chunk_lane(a.chunks, a.words, chunk, &count, &post_off);
        const bool valid = lane < count;
        const uint32_t tile = id >> kTileShift;
        const uint32_t prev = __shfl_up(tile, 1, 64);
        const bool head = valid && (lane == 0 || tile != prev);
        const uint64_t heads = __ballot(head);
        const uint64_t above = (lane == 63) ? 0ull : (heads & (~0ull << (lane + 1)));
        const int next = above ? (int)__builtin_ctzll(above) : count;
        const int run = next - lane;
        if (!place) {
            if (head) atomicAdd(&a.tile_cnt[tile], (uint32_t)run);
            continue;
        }
        // entry word x: the key's users range when the batch is one query group, else its
        // slot; the low five bits take the ad's offset in its tile
        uint32_t entry_x = u << kTileShift;
        if (a.users_off) {
            const uint32_t u0 = a.users_off[u];
            entry_x = (u0 << 13) | ((a.users_off[u + 1] - u0 - 1u) << kTileShift);
        }
        uint32_t base = 0;
        if (head) base = atomicAdd(&a.tile_fill[tile], (uint32_t)run);
        const uint64_t upto = (lane == 63) ? heads : (heads & ((2ull << lane) - 1ull));
        const int my_head = upto ? 63 - (int)__builtin_clzll(upto) : 0;
        base = __shfl(base, my_head, 64);
        if (valid) {
            const uint32_t pos = a.tile_off[tile] + base + (uint32_t)(lane - my_head);
            const float w = a.weights[post_off + lane];
            const int wfix = __double2int_rn(ldexp((double)w, a.uk_wshift[u]));
            reinterpret_cast<uint2*>(a.bucket)[pos] =
                make_uint2(entry_x | (id & (kTileAds - 1)), (uint32_t)wfix);
        }
    }
}

__global__ __launch_bounds__(64) void k_decode_key(const ChunkHdr* chunks, const uint32_t* words,
                                                   const float* weights, uint32_t chunk0,
                                                   uint32_t* ids, float* w) {
    const int lane = lane_id();
    const uint32_t chunk = chunk0 + blockIdx.x;
    int count;
    uint32_t post_off;
    const uint32_t id = decode_chunk_lane(chunks, words, chunk, &count, &post_off);
    if (lane < count) {
        const uint32_t out = blockIdx.x * kChunk + lane;
        ids[out] = id;
        w[out] = weights[post_off + lane];
    }
}

// ------------------------------------------------------------------ fused scoring

// One work-group (16 wavefronts) scores one 256-query group against a sequence of 32-ad
// tiles (persistent: tiles blockIdx.x, blockIdx.x + gridDim.x, ...). The waves specialise:
//   waves 0..7  (consumers) - wave w owns query rows [32w, 32w + 32). Per tile: read and
//                             clear its 32x32 block of the cross term, run the dot products
//                             on the matrix cores, add, select.
//   waves 8..15 (producers) - one tile ahead: stage the next tile's embedding block in LDS
//                             and accumulate its cross term into the other LDS buffer.
// Two barriers per tile hand the double-buffered accumulators and the embedding stage over.
//
// Embedding layout (FP32 copy): per 32-ad block, D/8 quads x 64 lanes x 4 floats, where
// quad i of lane l holds e[32b + (l & 31)][8i + 2j + (l >> 5)] for j = 0..3. Step s = 4i + j
// of the K loop then finds the B operand of v_mfma_f32_32x32x2_f32 (B[k][n] with
// k = l >> 5, n = l & 31) in component j of quad i.
//
// Accumulator layout of v_mfma_f32_32x32x2_f32: register r of lane l holds row
// 8 * (r >> 2) + 4 * (l >> 5) + (r & 3), column l & 31.
//
// Cross-term accumulators: int64 per (query, ad) in LDS, column swizzled by the query's low
// five bits so that the 32 users of one posting (same ad, 32 consecutive queries) and the
// 32 ads of one accumulator row both fall into distinct banks.
constexpr int kProducerWaves = 8;
constexpr int kLight = 8;  // entries with at most this many users are expanded per lane

// Queries per group: 256 (8 consumer waves) up to d = 64, 128 (4 consumer waves) above, so
// that the U operand and the LDS buffers fit.
template <int D> struct ScoreShape {
    static constexpr int GQ = D <= 64 ? 256 : 128;
    static constexpr int CW = GQ / 32;
    static constexpr int NT = 64 * (CW + kProducerWaves);
};

__device__ __forceinline__ int acc_idx(int q, int o) { return q * kTileAds + (o ^ (q & 31)); }

// Rare path of the selection epilogue: append one survivor to its query's candidate buffer.
// Kept out of line so that the per-row buffer addresses are not hoisted into registers.
__device__ __attribute__((noinline)) void append_candidate(unsigned long long* cand,
                                                           uint32_t* cand_cnt, int cap, int q,
                                                           uint32_t key, uint32_t idk) {
    const uint32_t pos = atomicAdd(&cand_cnt[q], 1u);
    if (pos < (uint32_t)cap)
        cand[(int64_t)q * cap + pos] = ((unsigned long long)key << 32) | (unsigned long long)idk;
}

// Dense test hook: store one (query, ad) pair of terms (out of line, as above).
__device__ __attribute__((noinline)) void store_dense(float* deep_out, float* wide_out,
                                                      int64_t idx, float deep, float wide) {
    deep_out[idx] = deep;
    wide_out[idx] = wide;
}

// Bucket entry: x = (u0 << 13) | ((cnt - 1) << 5) | ad offset when the batch is one query
// group (the key's users are users[u0, u0 + cnt)), else (slot << 5) | ad offset; y = w_fix.
// Producer wave pw owns entries beg + pw + 8 * (lane + 64 r) of each tile; round r = 0 is
// prefetched one tile ahead.
struct ProdTile {
    uint32_t beg, end;  // the tile's bucket range
    uint2 e0;           // this lane's round-0 entry (valid if beg + pw + 8 * lane < end)
};

__device__ __forceinline__ void cross_entries(const ScoreArgs& a, int g, uint2 e, bool valid,
                                              unsigned long long* acc) {
    const int lane = lane_id();
    const uint2* users = reinterpret_cast<const uint2*>(a.users);
    uint32_t cnt = 0, u0 = 0;
    if (valid) {
        if (a.packed) {
            u0 = e.x >> 13;
            cnt = ((e.x >> kTileShift) & 255u) + 1u;
        } else {
            const uint32_t slot = (e.x >> kTileShift) * (uint32_t)a.n_qgroups + (uint32_t)g;
            u0 = a.users_off[slot];
            cnt = a.users_off[slot + 1] - u0;
        }
    }
    const int o = (int)(e.x & (kTileAds - 1));
    const int w = (int)e.y;
    // light entries: each lane expands its own users (loads first, then the adds)
    if (cnt > 0 && cnt <= (uint32_t)kLight) {
        uint2 ue[kLight];
#pragma unroll
        for (int j = 0; j < kLight; ++j)
            if ((uint32_t)j < cnt) ue[j] = users[u0 + j];
#pragma unroll
        for (int j = 0; j < kLight; ++j)
            if ((uint32_t)j < cnt)
                atomicAdd(&acc[acc_idx((int)ue[j].x, o)],
                          (unsigned long long)((long long)(int)ue[j].y * (long long)w));
    }
    // heavy entries: the whole wave expands one entry's users at a time
    uint64_t heavy = __ballot(cnt > (uint32_t)kLight);
    while (heavy) {
        const int h = (int)__builtin_ctzll(heavy);
        heavy &= heavy - 1;
        const uint32_t hu0 = (uint32_t)__builtin_amdgcn_readlane((int)u0, h);
        const uint32_t hcnt = (uint32_t)__builtin_amdgcn_readlane((int)cnt, h);
        const int ho = __builtin_amdgcn_readlane(o, h);
        const int hw = __builtin_amdgcn_readlane(w, h);
        for (uint32_t j0 = 0; j0 < hcnt; j0 += 256) {
            uint2 ue[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t j = j0 + (uint32_t)(lane + 64 * r);
                if (j < hcnt) ue[r] = users[hu0 + j];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t j = j0 + (uint32_t)(lane + 64 * r);
                if (j < hcnt)
                    atomicAdd(&acc[acc_idx((int)ue[r].x, ho)],
                              (unsigned long long)((long long)(int)ue[r].y * (long long)hw));
            }
        }
    }
}

__device__ __forceinline__ uint2 prod_bounds(const ScoreArgs& a, uint32_t tile) {
    return make_uint2(a.tile_off[tile], a.tile_off[tile + 1]);
}

__device__ __forceinline__ ProdTile prod_entries(const ScoreArgs& a, uint2 b, int pw) {
    ProdTile t;
    t.beg = b.x;
    t.end = b.y;
    const uint32_t ei = t.beg + (uint32_t)pw + kProducerWaves * (uint32_t)lane_id();
    t.e0 = ei < t.end ? reinterpret_cast<const uint2*>(a.bucket)[ei] : make_uint2(0u, 0u);
    return t;
}

// Cross term of one tile (this wave's share), round 0 from the prefetched entry.
__device__ __forceinline__ void prod_tile(const ScoreArgs& a, int g, int pw, const ProdTile& t,
                                          unsigned long long* acc) {
    const int lane = lane_id();
    const uint2* bucket = reinterpret_cast<const uint2*>(a.bucket);
    constexpr uint32_t kRound = kProducerWaves * 64u;
    const uint32_t first = t.beg + (uint32_t)pw;
    if (first >= t.end) return;
    cross_entries(a, g, t.e0, first + kProducerWaves * (uint32_t)lane < t.end, acc);
    for (uint32_t base = first + kRound; base < t.end; base += kRound) {
        const uint32_t ei = base + kProducerWaves * (uint32_t)lane;
        const bool ok = ei < t.end;
        const uint2 e = ok ? bucket[ei] : make_uint2(0u, 0u);
        cross_entries(a, g, e, ok, acc);
    }
}

// Persistent over tiles blockIdx.x, blockIdx.x + gridDim.x, ...; iteration `it` has the
// consumers score tile it from LDS buffers [it & 1] (and clear the accumulators they read)
// while the producers fill buffers [(it + 1) & 1] with tile it + 1 and prefetch the entries
// of tile it + 2. Every wave executes exactly 1 + n_it barriers.
template <int D, int MODE>
__global__ __launch_bounds__(ScoreShape<D>::NT, 1) void k_score(ScoreArgs a) {
    constexpr int NQ = D / 8;  // quads per lane
    constexpr int GQ = ScoreShape<D>::GQ;
    constexpr int CW = ScoreShape<D>::CW;
    constexpr int NT = ScoreShape<D>::NT;
    constexpr int kProdThreads = 64 * kProducerWaves;
    __shared__ unsigned long long s_acc[2][GQ * kTileAds];
    __shared__ f32x4 s_emb[2][NQ * 64];
    __shared__ double s_inv[GQ];
    __shared__ float s_thr[GQ];
    __shared__ uint32_t s_thr_hi[GQ];
    __shared__ uint32_t s_thr_lo[GQ];
    __shared__ uint32_t s_live[GQ];

    const int tid = (int)threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const bool producer = wave >= CW;
    const int g = (int)blockIdx.y;
    const int qbase = g * GQ;
    const int B = a.n_queries;
    const int G = (int)gridDim.x;
    const int first = (int)blockIdx.x;
    if (first >= a.n_work) return;
    const int n_it = (a.n_work - first + G - 1) / G;

    for (int i = tid; i < 2 * GQ * kTileAds; i += NT) (&s_acc[0][0])[i] = 0ull;
    for (int i = tid; i < GQ; i += NT) {
        const int q = qbase + i;
        const bool in = q < B;
        s_inv[i] = in ? a.qinv[q] : 0.0;
        if (MODE == 0) {
            const uint32_t hi = in ? a.thresh[2 * q] : 0xffffffffu;
            s_thr_hi[i] = hi;
            s_thr_lo[i] = in ? a.thresh[2 * q + 1] : 0xffffffffu;
            s_thr[i] = key_score(hi);
            s_live[i] = (in && a.active[q]) ? 1u : 0u;
        } else {
            s_live[i] = in ? 1u : 0u;
        }
    }
    const f32x4* emb = reinterpret_cast<const f32x4*>(a.emb);
    auto tile_at = [&](int i) -> uint32_t {
        const int w = first + i * G;
        return a.tile_list ? a.tile_list[w] : (uint32_t)w;
    };
    __syncthreads();

    if (producer) {
        const int pw = wave - CW;
        const int ptid = tid - 64 * CW;
        // pipeline: bucket bounds two tiles ahead, round-0 entries one tile ahead
        const uint32_t t0 = tile_at(0);
        for (int j = ptid; j < NQ * 64; j += kProdThreads) s_emb[0][j] = emb[(int64_t)t0 * NQ * 64 + j];
        prod_tile(a, g, pw, prod_entries(a, prod_bounds(a, t0), pw), s_acc[0]);
        ProdTile p1{};
        uint2 b2 = make_uint2(0u, 0u);
        if (n_it > 1) p1 = prod_entries(a, prod_bounds(a, tile_at(1)), pw);
        if (n_it > 2) b2 = prod_bounds(a, tile_at(2));
        __syncthreads();
        for (int it = 0; it < n_it; ++it) {
            const int nb = (it & 1) ^ 1;
            if (it + 1 < n_it) {
                const uint32_t tn = tile_at(it + 1);
                for (int j = ptid; j < NQ * 64; j += kProdThreads)
                    s_emb[nb][j] = emb[(int64_t)tn * NQ * 64 + j];
                uint2 b3 = make_uint2(0u, 0u);
                if (it + 3 < n_it) b3 = prod_bounds(a, tile_at(it + 3));
                ProdTile p2{};
                if (it + 2 < n_it) p2 = prod_entries(a, b2, pw);
                prod_tile(a, g, pw, p1, s_acc[nb]);
                p1 = p2;
                b2 = b3;
            }
            __syncthreads();
        }
        return;
    }

    // consumer: A operand (user rows) of this wave's 32-query block, kept in registers
    const int q0 = qbase + wave * 32;
    float ureg[D / 2];
    {
        const int q = q0 + (lane & 31);
        const int kofs = lane >> 5;
#pragma unroll
        for (int s = 0; s < D / 2; ++s)
            ureg[s] = (q < B) ? a.user[(int64_t)q * D + 2 * s + kofs] : 0.0f;
    }
    bool wave_live = false;
    if (q0 < B) {
        uint32_t any = 0;
        for (int i = 0; i < 32; ++i) any |= s_live[wave * 32 + i];
        wave_live = any != 0;
    }
    __syncthreads();

    for (int it = 0; it < n_it; ++it) {
        const int cur = it & 1;
        unsigned long long* acc = s_acc[cur];
        if (!wave_live) {
            // rows no live wave reads: keep the buffer clear for its next use
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int ql = wave * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                acc[acc_idx(ql, lane & 31)] = 0ull;
            }
        } else {
            const uint32_t tile = tile_at(it);
            f32x16 c = {};
            const f32x4* eb = s_emb[cur];
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                const f32x4 e4 = eb[i * 64 + lane];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    c = __builtin_amdgcn_mfma_f32_32x32x2f32(ureg[4 * i + j], e4[j], c, 0, 0, 0);
            }
            const int64_t ad = (int64_t)tile * kTileAds + (lane & 31);
            const bool ad_ok = ad < a.n_ads;
            uint32_t* skeys = nullptr;
            uint32_t scol = 0;
            if (MODE == 1) {
                skeys = a.sample_keys + (int64_t)q0 * a.sample_ld;
                scol = (uint32_t)(first + it * G) * kTileAds + (uint32_t)(lane & 31);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int ql = wave * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int q = qbase + ql;
                const int idx = acc_idx(ql, lane & 31);
                const long long v = (long long)acc[idx];
                acc[idx] = 0ull;
                const float wide = (float)((double)v * s_inv[ql]);
                const float deep = c[r];
                if (MODE == 2) {
                    if (ad_ok && q < B)
                        store_dense(a.deep_out, a.wide_out, (int64_t)q * a.n_ads + ad, deep, wide);
                } else {
                    const float sc = deep + wide;
                    if (MODE == 1) {
                        // row base of this wave's 32-query block + a 32-bit offset per row
                        if (q < B)
                            skeys[(uint32_t)(ql - wave * 32) * (uint32_t)a.sample_ld + scol] =
                                ad_ok ? score_key(sc) : 0u;
                    } else if (ad_ok && sc >= s_thr[ql] && s_live[ql]) {
                        // rare: exact (key, id) comparison against the threshold
                        const uint32_t key = score_key(sc);
                        const uint32_t idk = 0xffffffffu - (uint32_t)ad;
                        if (key > s_thr_hi[ql] || (key == s_thr_hi[ql] && idk >= s_thr_lo[ql]))
                            append_candidate(a.cand, a.cand_cnt, a.cap, q, key, idk);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ threshold select

// Per query q (one block): the j-th largest of the n_cols sample keys (1-based j = jq[q]),
// found by three radix passes of 11 + 11 + 10 bits over LDS histograms.
__global__ __launch_bounds__(1024) void k_select(SelectArgs a) {
    __shared__ uint32_t hist[2048];
    __shared__ uint32_t sbuf[1024 / 64 + 1];
    __shared__ uint32_t s_res[2];
    const int q = (int)blockIdx.x;
    const int tid = (int)threadIdx.x;
    if (a.only_status >= 0 && a.status[q] != a.only_status) return;
    if (a.kq[q] <= 0) return;
    const int64_t j = a.jq[q];
    if (j > a.n_cols || j <= 0) {
        if (tid == 0) { a.thresh[2 * q] = 0u; a.thresh[2 * q + 1] = 0u; }
        return;
    }
    const uint32_t* row = a.keys + (int64_t)q * a.ld;
    uint32_t prefix = 0, mask = 0, rem = (uint32_t)j;
    const int shifts[3] = {21, 10, 0};
    const int widths[3] = {11, 11, 10};
    for (int p = 0; p < 3; ++p) {
        const int sh = shifts[p], nb = 1 << widths[p];
        for (int i = tid; i < 2048; i += 1024) hist[i] = 0;
        __syncthreads();
        for (int64_t i = tid; i < a.n_cols; i += 1024) {
            const uint32_t x = row[i];
            if ((x & mask) == prefix) atomicAdd(&hist[(x >> sh) & (nb - 1)], 1u);
        }
        __syncthreads();
        // thread t covers bins nb-1-2t and nb-2-2t (descending); scan from the top
        const int b0 = nb - 1 - 2 * tid, b1 = nb - 2 - 2 * tid;
        const uint32_t h0 = (b0 >= 0) ? hist[b0] : 0u, h1 = (b1 >= 0) ? hist[b1] : 0u;
        uint32_t tot;
        const uint32_t above = block_excl_scan<1024>(h0 + h1, sbuf, &tot);
        if (b0 >= 0 && above < rem && rem <= above + h0) { s_res[0] = (uint32_t)b0; s_res[1] = above; }
        if (b1 >= 0 && above + h0 < rem && rem <= above + h0 + h1) {
            s_res[0] = (uint32_t)b1;
            s_res[1] = above + h0;
        }
        __syncthreads();
        prefix |= s_res[0] << sh;
        mask |= (uint32_t)(nb - 1) << sh;
        rem -= s_res[1];
        __syncthreads();
    }
    if (tid == 0) { a.thresh[2 * q] = prefix; a.thresh[2 * q + 1] = 0u; }
}

// ------------------------------------------------------------------ finalize

__global__ __launch_bounds__(1024) void k_finalize(FinalArgs a) {
    __shared__ unsigned long long s[kCandCap];
    const int q = (int)blockIdx.x;
    const int tid = (int)threadIdx.x;
    if (!a.active[q]) return;
    const int K = a.kq[q];
    const uint32_t c = a.cand_cnt[q];
    if ((int64_t)c < (int64_t)K) {
        if (tid == 0) { a.status[q] = kStatusNeedLower; atomicAdd(a.unresolved, 1u); }
        return;
    }
    const int n = (int)min(c, (uint32_t)a.cap);
    int P = 64;
    while (P < n) P <<= 1;
    const unsigned long long* src = a.cand + (int64_t)q * a.cap;
    for (int i = tid; i < P; i += 1024) s[i] = (i < n) ? src[i] : 0ull;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < P; i += 1024) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const unsigned long long x = s[i], y = s[ixj];
                    const bool desc = (i & k) == 0;
                    if (desc ? (x < y) : (x > y)) { s[i] = y; s[ixj] = x; }
                }
            }
            __syncthreads();
        }
    }
    if (c > (uint32_t)a.cap) {
        if (tid == 0) {
            const unsigned long long t = s[K - 1];
            a.thresh[2 * q] = (uint32_t)(t >> 32);
            a.thresh[2 * q + 1] = (uint32_t)t;
            a.status[q] = kStatusOverflow;
            atomicAdd(a.unresolved, 1u);
        }
        return;
    }
    const int64_t o = a.out_off[q];
    for (int i = tid; i < K; i += 1024) {
        const unsigned long long t = s[i];
        a.out_ids[o + i] = 0xffffffffu - (uint32_t)t;
        a.out_scores[o + i] = key_score((uint32_t)(t >> 32));
    }
    if (tid == 0) { a.status[q] = kStatusDone; a.active[q] = 0u; }
}

// ------------------------------------------------------------------ launchers

static int last(hipError_t e) { return e == hipSuccess ? (int)hipGetLastError() : (int)e; }

int launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, void* stream) {
    if (n <= 0) return 0;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, p, v, n);
    return last(hipSuccess);
}

int64_t scan_tmp_words(int64_t n) { return (n + kScanBlock) / kScanBlock + 1; }

int launch_excl_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    // blocks cover n + 1 outputs (the last one is the total)
    const int64_t nb = (n + 1 + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanNT), 0, st, in, n, tmp);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, tmp, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanNT), 0, st, in, n, tmp, out);
    return last(hipSuccess);
}

int launch_decode(const DecodeArgs& a, int place, void* stream) {
    if (a.total_chunks == 0) return 0;
    const uint32_t waves = (a.total_chunks + kChunksPerWave - 1) / kChunksPerWave;
    const unsigned blocks = (waves + 3u) / 4u;
    hipLaunchKernelGGL(k_decode, dim3(blocks), dim3(256), 0, (hipStream_t)stream, a, place);
    return last(hipSuccess);
}

int launch_decode_key(const ChunkHdr* chunks, const uint32_t* words, const float* weights,
                      uint32_t chunk0, uint32_t n_chunks, uint32_t* ids, float* w, void* stream) {
    if (n_chunks == 0) return 0;
    hipLaunchKernelGGL(k_decode_key, dim3(n_chunks), dim3(64), 0, (hipStream_t)stream, chunks,
                       words, weights, chunk0, ids, w);
    return last(hipSuccess);
}

template <int D>
static void launch_score_d(const ScoreArgs& a, int mode, dim3 grid, hipStream_t st) {
    constexpr int NT = ScoreShape<D>::NT;
    if (mode == 0) hipLaunchKernelGGL((k_score<D, 0>), grid, dim3(NT), 0, st, a);
    else if (mode == 1) hipLaunchKernelGGL((k_score<D, 1>), grid, dim3(NT), 0, st, a);
    else hipLaunchKernelGGL((k_score<D, 2>), grid, dim3(NT), 0, st, a);
}

int score_group_queries(int dim) { return dim <= 64 ? 256 : 128; }

bool score_dim_supported(int dim) {
    switch (dim) {
        case 16: case 32: case 48: case 64: case 80: case 96: case 112: case 128: return true;
        default: return false;
    }
}

int launch_score(const ScoreArgs& a, int dim, int mode, int ctas, void* stream) {
    if (a.n_work <= 0 || a.n_qgroups <= 0) return 0;
    const int c = a.n_work < ctas ? a.n_work : ctas;
    dim3 grid((unsigned)c, (unsigned)a.n_qgroups);
    hipStream_t st = (hipStream_t)stream;
    switch (dim) {
        case 16: launch_score_d<16>(a, mode, grid, st); break;
        case 32: launch_score_d<32>(a, mode, grid, st); break;
        case 48: launch_score_d<48>(a, mode, grid, st); break;
        case 64: launch_score_d<64>(a, mode, grid, st); break;
        case 80: launch_score_d<80>(a, mode, grid, st); break;
        case 96: launch_score_d<96>(a, mode, grid, st); break;
        case 112: launch_score_d<112>(a, mode, grid, st); break;
        case 128: launch_score_d<128>(a, mode, grid, st); break;
        default: return (int)hipErrorInvalidValue;
    }
    return last(hipSuccess);
}

int launch_select(const SelectArgs& a, int n_queries, void* stream) {
    if (n_queries <= 0) return 0;
    hipLaunchKernelGGL(k_select, dim3((unsigned)n_queries), dim3(1024), 0, (hipStream_t)stream, a);
    return last(hipSuccess);
}

int launch_finalize(const FinalArgs& a, int n_queries, void* stream) {
    if (n_queries <= 0) return 0;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)n_queries), dim3(1024), 0, (hipStream_t)stream, a);
    return last(hipSuccess);
}

}  // namespace ebr
