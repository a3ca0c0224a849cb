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
// The cross term of Section 3.3 (equation "hitmatch") is accumulated as 64-bit fixed point
// with a per-query scale 2^S chosen on the host so that the sum cannot overflow: every
// product m*w (exact in FP64) is rounded once to an integer multiple of 2^-S and the sum is
// exact, so the result does not depend on the order in which postings are added. Scores are
// therefore bit-identical across passes, tile schedules and batch compositions.
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

__global__ __launch_bounds__(256) void k_decode(DecodeArgs a, int place) {
    const int lane = lane_id();
    const uint32_t gw = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (gw >= a.total_chunks) return;
    // distinct-key slot owning this chunk: the last u with prefix[u] <= gw
    int lo = 0, hi = a.n_ukeys;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (a.uk_chunk_prefix[mid] <= gw) lo = mid; else hi = mid;
    }
    const uint32_t u = (uint32_t)lo;
    const uint32_t chunk = a.uk_chunk_begin[u] + (gw - a.uk_chunk_prefix[u]);
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
        return;
    }
    uint32_t base = 0;
    if (head) base = atomicAdd(&a.tile_fill[tile], (uint32_t)run);
    const uint64_t upto = (lane == 63) ? heads : (heads & ((2ull << lane) - 1ull));
    const int my_head = upto ? 63 - (int)__builtin_clzll(upto) : 0;
    base = __shfl(base, my_head, 64);
    if (valid) {
        const uint32_t pos = a.tile_off[tile] + base + (uint32_t)(lane - my_head);
        const float w = a.weights[post_off + lane];
        reinterpret_cast<uint2*>(a.bucket)[pos] =
            make_uint2((u << kTileShift) | (id & (kTileAds - 1)), __float_as_uint(w));
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

// One work-group = 8 wavefronts = 256 queries (one query group) x one 32-ad tile at a time.
// Wave w owns query rows [32w, 32w + 32) of the group.
//
// Embedding layout (FP32 copy): per 32-ad block, D/8 quads x 64 lanes x 4 floats, where
// quad i of lane l holds e[32b + (l & 31)][8i + 2j + (l >> 5)] for j = 0..3. Step s = 4i + j
// of the K loop then finds the B operand of v_mfma_f32_32x32x2_f32 (B[k][n] with
// k = l >> 5, n = l & 31) in component j of quad i, and a wave loads the whole block with
// D/8 fully coalesced 1 KiB loads.
//
// Accumulator layout of v_mfma_f32_32x32x2_f32: register r of lane l holds row
// 8 * (r >> 2) + 4 * (l >> 5) + (r & 3), column l & 31.
constexpr int kScoreNT = 512;

template <int D, int MODE>
__global__ __launch_bounds__(kScoreNT, (D <= 64 ? 4 : 2)) void k_score(ScoreArgs a) {
    constexpr int NQ = D / 8;  // quads per lane
    __shared__ unsigned long long s_acc[kGroupQueries * kTileAds];  // 64 KiB
    __shared__ uint32_t s_pre[kScoreNT + 1];
    __shared__ uint32_t s_uoff[kScoreNT];
    __shared__ uint32_t s_ent[kScoreNT];
    __shared__ float s_w[kScoreNT];
    __shared__ double s_scale[kGroupQueries];
    __shared__ double s_inv[kGroupQueries];
    __shared__ uint32_t s_thr_hi[kGroupQueries];
    __shared__ uint32_t s_thr_lo[kGroupQueries];
    __shared__ uint32_t s_live[kGroupQueries];
    __shared__ uint32_t s_scan[kScoreNT / 64 + 1];

    const int tid = (int)threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const int g = (int)blockIdx.y;
    const int qbase = g * kGroupQueries;
    const int B = a.n_queries;

    for (int i = tid; i < kGroupQueries * kTileAds; i += kScoreNT) s_acc[i] = 0ull;
    for (int i = tid; i < kGroupQueries; i += kScoreNT) {
        const int q = qbase + i;
        const bool in = q < B;
        s_scale[i] = in ? a.qscale[q] : 0.0;
        s_inv[i] = in ? a.qinv[q] : 0.0;
        if (MODE == 0) {
            s_thr_hi[i] = in ? a.thresh[2 * q] : 0xffffffffu;
            s_thr_lo[i] = in ? a.thresh[2 * q + 1] : 0xffffffffu;
            s_live[i] = (in && a.active[q]) ? 1u : 0u;
        } else {
            s_live[i] = in ? 1u : 0u;
        }
    }

    // A operand (user rows) for this wave's 32-query block, kept in registers.
    const int q0 = qbase + wave * 32;
    const bool wave_rows = q0 < B;
    float ureg[D / 2];
    {
        const int q = q0 + (lane & 31);
        const int kofs = lane >> 5;
#pragma unroll
        for (int s = 0; s < D / 2; ++s)
            ureg[s] = (q < B) ? a.user[(int64_t)q * D + 2 * s + kofs] : 0.0f;
    }
    __syncthreads();
    bool wave_live = false;
    if (wave_rows) {
        uint32_t any = 0;
        for (int i = 0; i < 32; ++i) any |= s_live[wave * 32 + i];
        wave_live = any != 0;
    }

    const f32x4* emb = reinterpret_cast<const f32x4*>(a.emb);
    const uint2* bucket = reinterpret_cast<const uint2*>(a.bucket);
    const uint2* users = reinterpret_cast<const uint2*>(a.users);
    const int n_qg = a.n_qgroups;

    for (int w = (int)blockIdx.x; w < a.n_work; w += (int)gridDim.x) {
        const uint32_t tile = a.tile_list ? a.tile_list[w] : (uint32_t)w;

        // B operand: this tile's embedding block (issued early, consumed after the cross term)
        f32x4 ereg[NQ];
        if (wave_live) {
            const f32x4* src = emb + (int64_t)tile * NQ * 64 + lane;
#pragma unroll
            for (int i = 0; i < NQ; ++i) ereg[i] = src[i * 64];
        }

        // ---- cross term: the tile's bucket entries times each entry's key users
        const uint32_t beg = a.tile_off[tile], end = a.tile_off[tile + 1];
        for (uint32_t base = beg; base < end; base += kScoreNT) {
            const uint32_t i = base + (uint32_t)tid;
            uint32_t cnt = 0;
            if (i < end) {
                const uint2 e = bucket[i];
                const uint32_t slot = (e.x >> kTileShift) * (uint32_t)n_qg + (uint32_t)g;
                const uint32_t u0 = a.users_off[slot];
                cnt = a.users_off[slot + 1] - u0;
                s_uoff[tid] = u0;
                s_ent[tid] = e.x & (kTileAds - 1);
                s_w[tid] = __uint_as_float(e.y);
            }
            uint32_t total;
            const uint32_t pre = block_excl_scan<kScoreNT>(cnt, s_scan, &total);
            s_pre[tid] = pre;
            const int n_here = (int)min((uint32_t)kScoreNT, end - base);
            if (tid == 0) s_pre[n_here] = total;
            __syncthreads();
            for (uint32_t x = (uint32_t)tid; x < total; x += kScoreNT) {
                int lo = 0, hi = n_here;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_pre[mid] <= x) lo = mid; else hi = mid;
                }
                const uint2 ue = users[s_uoff[lo] + (x - s_pre[lo])];
                const int ql = (int)ue.x;
                const double prod = (double)__uint_as_float(ue.y) * (double)s_w[lo];
                const long long v = __double2ll_rn(prod * s_scale[ql]);
                atomicAdd(&s_acc[ql * kTileAds + (int)s_ent[lo]], (unsigned long long)v);
            }
            __syncthreads();
        }

        // ---- this wave's 32 x 32 block of the cross term, then clear it for the next tile
        float wide[16];
        if (wave_live) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int ql = wave * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int idx = ql * kTileAds + (lane & 31);
                const long long v = (long long)s_acc[idx];
                s_acc[idx] = 0ull;
                wide[r] = (float)((double)v * s_inv[ql]);
            }
        }
        __syncthreads();
        if (!wave_live) continue;

        // ---- dot products on the matrix cores
        f32x16 c = {};
#pragma unroll
        for (int s = 0; s < D / 2; ++s)
            c = __builtin_amdgcn_mfma_f32_32x32x2f32(ureg[s], ereg[s >> 2][s & 3], c, 0, 0, 0);

        // ---- epilogue
        const int64_t ad = (int64_t)tile * kTileAds + (lane & 31);
        const bool ad_ok = ad < a.n_ads;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int ql = wave * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int q = qbase + ql;
            const float deep = c[r];
            if (MODE == 2) {
                if (ad_ok && q < B) {
                    a.deep_out[(int64_t)q * a.n_ads + ad] = deep;
                    a.wide_out[(int64_t)q * a.n_ads + ad] = wide[r];
                }
            } else {
                const float sc = deep + wide[r];
                const uint32_t key = score_key(sc);
                if (MODE == 1) {
                    if (q < B)
                        a.sample_keys[(int64_t)q * a.sample_ld + (int64_t)w * kTileAds + (lane & 31)] =
                            ad_ok ? key : 0u;
                } else {
                    if (ad_ok && key >= s_thr_hi[ql] && s_live[ql]) {
                        const uint32_t idk = 0xffffffffu - (uint32_t)ad;
                        if (key > s_thr_hi[ql] || idk >= s_thr_lo[ql]) {
                            const uint32_t pos = atomicAdd(&a.cand_cnt[q], 1u);
                            if (pos < (uint32_t)a.cap)
                                a.cand[(int64_t)q * a.cap + pos] =
                                    ((unsigned long long)key << 32) | (unsigned long long)idk;
                        }
                    }
                }
            }
        }
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
    const unsigned blocks = (a.total_chunks + 3u) / 4u;
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
    if (mode == 0) hipLaunchKernelGGL((k_score<D, 0>), grid, dim3(kScoreNT), 0, st, a);
    else if (mode == 1) hipLaunchKernelGGL((k_score<D, 1>), grid, dim3(kScoreNT), 0, st, a);
    else hipLaunchKernelGGL((k_score<D, 2>), grid, dim3(kScoreNT), 0, st, a);
}

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
