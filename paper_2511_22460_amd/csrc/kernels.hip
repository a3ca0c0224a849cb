// gfx950 (CDNA4) kernels of libebr.
//
// One batch of queries runs as:
//   0. k_chunk_map       - per chunk of the batch's distinct keys, its key slot and index
//                          chunk.
//   1. k_decode (count)  - every chunk is decoded by one wavefront (eight chunks' loads in
//                          flight together); postings are counted per super-tile (2048
//                          ads; 1024 with split buckets).
//   2. scan              - exclusive scan of the super-tile counts.
//   3. k_decode (place)  - decode again and place each posting (key slot, ad, weight) into
//                          its super-tile's staging range.
//   3b. k_refine         - per super-tile, a counting sort by 32-ad tile in LDS: the batch's
//                          postings, tile-major (the bucket).
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
// The cross term of Section 3.3 (equation "hitmatch") is accumulated in fixed point. Each
// posting weight of key k is scaled exactly to w' = w * 2^Sw_k (|w'| < 2^30) when it is placed
// into its bucket, and each (query, key) multiplier on the host to m' = m * 2^(S_q - Sw_k), so
// that m' * w' = m * w * 2^S_q at one per-query scale with sum_j |m_j| max|W_kj| 2^S_q below
// 2^31 (32-bit cells) or 2^63 (64-bit cells). A (query, posting) pair adds round(fl(m' * w'))
// to its cell; the integer sum is exact and does not depend on the order of the adds, so
// scores are bit-identical across passes, tile schedules and batch compositions. A query whose
// 32-bit quantum is coarse against its returned scores is rerun with 64-bit cells.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "device_util.h"

namespace ebr {

template <int D> void launch_score_d(const ScoreArgs& a, int mode, int dt, dim3 grid, hipStream_t st);
template <int D> void launch_rescore_d(const RescoreArgs& a, int n_queries, hipStream_t st);
#define EBR_WIDTHS(X) X(16) X(32) X(48) X(64) X(80) X(96) X(112) X(128)
#define EBR_DECL(D)                                                                              \
    extern template void launch_score_d<D>(const ScoreArgs&, int, int, dim3, hipStream_t);      \
    extern template void launch_rescore_d<D>(const RescoreArgs&, int, hipStream_t);
EBR_WIDTHS(EBR_DECL)
#undef EBR_DECL

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

// One wavefront per distinct key of the batch: for each of the key's chunks, in batch order
// (chunk gc = uk_chunk_prefix[u] + i), its slot u and its chunk index in the index.
__global__ __launch_bounds__(256) void k_chunk_map(DecodeArgs a) {
    const int lane = lane_id();
    const int u = (int)(blockIdx.x * 4u + (threadIdx.x >> 6));
    if (u >= a.n_ukeys) return;
    const uint32_t p0 = a.uk_chunk_prefix[u], p1 = a.uk_chunk_prefix[u + 1];
    const uint32_t c0 = a.uk_chunk_begin[u];
    for (uint32_t gc = p0 + (uint32_t)lane; gc < p1; gc += 64u)
        a.chunk_map[gc] = make_uint2((uint32_t)u, c0 + (gc - p0));
}

// Chunks whose loads one decode wavefront issues together (headers, then every gap word and
// weight of the group), so that a group costs one chain of dependent loads.
constexpr int kDecGroup = 8;

// One wavefront decodes a.chunks_per_wave consecutive chunks of the batch's distinct keys and
// counts (place == 0) or places (place == 1) their postings into super-tile buckets of
// 2^sshift ads. Runs of postings in the same super-tile are aggregated into one atomic per run.
// A placed entry is ((slot << sshift) | ad mod 2^sshift, w' bits); k_refine orders each
// super-tile by 32-ad tile.
__global__ __launch_bounds__(256) void k_decode(DecodeArgs a, int place) {
    const int lane = lane_id();
    const uint32_t gw = blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t c_begin = gw * a.chunks_per_wave;
    if (c_begin >= a.total_chunks) return;
    const uint32_t c_end = min(a.total_chunks, c_begin + a.chunks_per_wave);
    for (uint32_t g0 = c_begin; g0 < c_end; g0 += kDecGroup) {
        const int n = (int)min((uint32_t)kDecGroup, c_end - g0);
        // lane i < n: chunk g0 + i's slot and index chunk, then its header
        uint2 m = make_uint2(0u, 0u);
        uint4 h = make_uint4(0u, 0u, 0u, 0u);
        if (lane < n) {
            m = a.chunk_map[g0 + (uint32_t)lane];
            h = *reinterpret_cast<const uint4*>(a.chunks + m.y);
        }
        // every chunk's gap words (and weights) for this lane, loads in flight together
        uint32_t lo[kDecGroup], hi[kDecGroup];
        float wt[kDecGroup];
        #pragma unroll
        for (int i = 0; i < kDecGroup; ++i) {
            lo[i] = hi[i] = 0u;
            wt[i] = 0.0f;
            if (i < n) {  // wave-uniform
                const uint32_t info = (uint32_t)__builtin_amdgcn_readlane((int)h.y, i);
                const uint32_t woff = (uint32_t)__builtin_amdgcn_readlane((int)h.z, i);
                const uint32_t poff = (uint32_t)__builtin_amdgcn_readlane((int)h.w, i);
                const int b = (int)(info & 63u), count = (int)((info >> 8) & 127u);
                if (lane >= 1 && lane < count && b > 0) {
                    const uint32_t* w = a.words + woff + (((uint32_t)(lane - 1) * (uint32_t)b) >> 5);
                    lo[i] = w[0];
                    hi[i] = w[1];
                }
                if (place && lane < count) wt[i] = a.weights ? a.weights[poff + (uint32_t)lane] : 1.0f;
            }
        }
        #pragma unroll
        for (int i = 0; i < kDecGroup; ++i) {
            if (i >= n) break;
            const uint32_t first = (uint32_t)__builtin_amdgcn_readlane((int)h.x, i);
            const uint32_t info = (uint32_t)__builtin_amdgcn_readlane((int)h.y, i);
            const uint32_t u = (uint32_t)__builtin_amdgcn_readlane((int)m.x, i);
            const int b = (int)(info & 63u), count = (int)((info >> 8) & 127u);
            uint32_t gap = 0;
            if (lane >= 1 && lane < count && b > 0) {
                const uint32_t sh = ((uint32_t)(lane - 1) * (uint32_t)b) & 31u;
                const uint64_t v = (((uint64_t)hi[i] << 32) | (uint64_t)lo[i]) >> sh;
                gap = (b == 32) ? (uint32_t)v : ((uint32_t)v & ((1u << b) - 1u));
            }
            const uint32_t delta = (lane >= 1 && lane < count) ? gap + 1u : 0u;
            const uint32_t id = first + wave_incl_scan(delta);
            const bool valid = lane < count;
            const uint32_t st = id >> a.sshift;
            const uint32_t prev = __shfl_up(st, 1, 64);
            const bool head = valid && (lane == 0 || st != prev);
            const uint64_t heads = __ballot(head);
            const uint64_t above = (lane == 63) ? 0ull : (heads & (~0ull << (lane + 1)));
            const int next = above ? (int)__builtin_ctzll(above) : count;
            const int run = next - lane;
            // a cold key of split buckets: each posting is placed once per user of the key
            const bool cold = (int)u >= a.cold_first;
            uint32_t c0 = 0, nusers = 1;
            if (cold) {
                c0 = a.cold_off[u - (uint32_t)a.cold_first];
                nusers = a.cold_off[u - (uint32_t)a.cold_first + 1] - c0;
            }
            if (!place) {
                if (head) atomicAdd(&a.st_cnt[st], (uint32_t)run * nusers);
                continue;
            }
            uint32_t base = 0;
            if (head) base = atomicAdd(&a.st_fill[st], (uint32_t)run * nusers);
            const uint64_t upto = (lane == 63) ? heads : (heads & ((2ull << lane) - 1ull));
            const int my_head = upto ? 63 - (int)__builtin_clzll(upto) : 0;
            base = __shfl(base, my_head, 64);
            if (valid) {
                const uint32_t pos = a.st_off[st] + base + (uint32_t)(lane - my_head) * nusers;
                const float ws = ldexpf(wt[i], a.uk_wshift[u]);  // exact: a power-of-two scale
                uint2* out = reinterpret_cast<uint2*>(a.stage) + pos;
                if (!cold) {
                    out[0] = make_uint2((u << a.sshift) | (id & ((1u << a.sshift) - 1u)), __float_as_uint(ws));
                } else {
                    // the pair's term round(fl(m' w')): an FP32 value that is an integer (split
                    // buckets: 1024-ad super-tiles)
                    const uint2* cu = reinterpret_cast<const uint2*>(a.cold_users) + c0;
                    const uint32_t gmask = (1u << a.gq_shift) - 1u;
                    for (uint32_t j = 0; j < nusers; ++j) {
                        const uint2 r = cu[j];
                        const float v = rintf(__uint_as_float(r.y) * ws);
                        out[j] = make_uint2(0x80000000u | ((r.x >> a.gq_shift) << 18) | ((r.x & gmask) << kSuperShift) |
                                                (id & (kSuperAds - 1)),
                                            __float_as_uint(v));
                    }
                }
            }
        }
    }
}

// Entries of one super-tile a k_refine work-group keeps in registers (per thread) when they
// fit; larger super-tiles are read twice.
constexpr int kRefineNT = 1024, kRefineRegs = 16;
constexpr int kRefineBins = std::max(kTilesPerSuper * (kSplitMaxGroups + 2), 1 << (kMaxSuperShift - kTileShift));
static_assert(kRefineBins <= 2 * kRefineNT, "two bins per thread in the offset scan");

// One work-group per super-tile: counting sort of its entries by (32-ad tile, sub-range)
// (LDS counters; one sub-range unless the buckets are split), the tile offsets, and the final
// entry format read by k_score: x = (u0 << 13) | ((cnt - 1) << 5) | ad & 31 when the batch is
// one query group (users[u0, u0 + cnt) are the key's users), (query row << 5) | ad & 31 for
// a cold pair (y: its term), else (slot << 5) | ad & 31; y = the bits of w'.
__global__ __launch_bounds__(kRefineNT) void k_refine(DecodeArgs a) {
    __shared__ uint32_t s_cnt[kRefineBins], s_off[kRefineBins];
    __shared__ uint32_t s_scan[kRefineNT / 64 + 1];
    const uint32_t st = blockIdx.x;
    const uint32_t beg = a.st_off[st], end = a.st_off[st + 1];
    const int tid = (int)threadIdx.x;
    const int tps = 1 << (a.sshift - kTileShift);  // tiles per super-tile
    const int S = a.n_sub, nb = tps * S;
    for (int b = tid; b < nb; b += kRefineNT) s_cnt[b] = 0u;
    __syncthreads();
    const uint2* in = reinterpret_cast<const uint2*>(a.stage);
    const bool regs = end - beg <= (uint32_t)(kRefineNT * kRefineRegs);
    uint2 e[kRefineRegs];
    // bin: tile within the super-tile, then sub-range: hot, warm, cold pairs of group g
    auto bin_of = [&](uint2 v) -> uint32_t {
        const uint32_t t = (v.x >> kTileShift) & (uint32_t)(tps - 1);
        if (S == 1) return t;
        const uint32_t sub = (v.x >> 31) ? 2u + ((v.x >> 18) & 0x1fffu)
                                          : ((v.x >> a.sshift) < (uint32_t)a.n_hot ? 0u : 1u);
        return t * (uint32_t)S + sub;
    };
    if (regs) {
        #pragma unroll
        for (int r = 0; r < kRefineRegs; ++r) {
            const uint32_t i = beg + (uint32_t)tid + (uint32_t)(r * kRefineNT);
            if (i < end) e[r] = in[i];
        }
        #pragma unroll
        for (int r = 0; r < kRefineRegs; ++r)
            if (beg + (uint32_t)tid + (uint32_t)(r * kRefineNT) < end) atomicAdd(&s_cnt[bin_of(e[r])], 1u);
    } else {
        for (uint32_t i = beg + (uint32_t)tid; i < end; i += kRefineNT) atomicAdd(&s_cnt[bin_of(in[i])], 1u);
    }
    __syncthreads();
    {
        // exclusive scan of the bin counts, two bins per thread
        const uint32_t c0 = 2 * tid < nb ? s_cnt[2 * tid] : 0u;
        const uint32_t c1 = 2 * tid + 1 < nb ? s_cnt[2 * tid + 1] : 0u;
        uint32_t tot;
        const uint32_t x = block_excl_scan<kRefineNT>(c0 + c1, s_scan, &tot);
        if (2 * tid < nb) { s_off[2 * tid] = beg + x; s_cnt[2 * tid] = 0u; }
        if (2 * tid + 1 < nb) { s_off[2 * tid + 1] = beg + x + c0; s_cnt[2 * tid + 1] = 0u; }
    }
    __syncthreads();
    for (int b = tid; b < nb; b += kRefineNT) {
        const uint64_t tile = (uint64_t)st * (uint64_t)tps + (uint64_t)(b / S);
        if (tile < (uint64_t)a.n_tiles) a.tile_off[tile * (uint64_t)S + (uint64_t)(b % S)] = s_off[b];
    }
    if (st == gridDim.x - 1 && tid == 0) a.tile_off[(uint64_t)a.n_tiles * (uint64_t)S] = end;
    uint2* out = reinterpret_cast<uint2*>(a.bucket);
    auto place = [&](uint2 v) {
        const uint32_t b = bin_of(v);
        const uint32_t pos = s_off[b] + atomicAdd(&s_cnt[b], 1u);
        const uint32_t u = v.x >> a.sshift, o = v.x & (kTileAds - 1);
        uint32_t x = (u << kTileShift) | o;
        if (S > 1 && (v.x >> 31)) {
            x = (((v.x >> kSuperShift) & 255u) << kTileShift) | o;  // cold pair: its query row
        } else if (a.users_off) {
            const uint32_t u0 = a.users_off[u];
            x = (u0 << 13) | ((a.users_off[u + 1] - u0 - 1u) << kTileShift) | o;
        }
        out[pos] = make_uint2(x, v.y);
    };
    if (regs) {
        #pragma unroll
        for (int r = 0; r < kRefineRegs; ++r)
            if (beg + (uint32_t)tid + (uint32_t)(r * kRefineNT) < end) place(e[r]);
    } else {
        for (uint32_t i = beg + (uint32_t)tid; i < end; i += kRefineNT) place(in[i]);
    }
}

// Decode chunk `chunk` (test hook path): returns this lane's id (lanes >= count return
// garbage).
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

// One wavefront per chunk of a run of consecutive keys: posting t of the run (in key order) goes
// to ids[t] / w[t]; an index without stored weights (unit weights) writes 1.
__global__ __launch_bounds__(64) void k_decode_key(const ChunkHdr* chunks, const uint32_t* words,
                                                   const float* weights, uint32_t chunk0,
                                                   uint32_t post_base, uint32_t* ids, float* w) {
    const int lane = lane_id();
    const uint32_t chunk = chunk0 + blockIdx.x;
    int count;
    uint32_t post_off;
    const uint32_t id = decode_chunk_lane(chunks, words, chunk, &count, &post_off);
    if (lane < count) {
        const uint32_t out = post_off - post_base + (uint32_t)lane;
        ids[out] = id;
        w[out] = weights ? weights[post_off + lane] : 1.0f;
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
    if (a.gate && *a.gate == 0u) return;
    if (a.ctl && a.ctl->error) return;
    if (a.only_status >= 0 && a.status[q] != a.only_status) return;
    if (a.kq[q] <= 0) return;
    int64_t j = a.jq[q];
    if (a.round == 1) j = a.kcnt[q] <= a.n_valid ? a.kcnt[q] : a.n_valid + 1;
    else if (a.round >= 2) j = a.n_valid + 1;
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

// Per query (one work-group): the candidate keys (score key << 32 | ~id) are sorted in LDS;
// with C candidates and a target of Kc = kcnt[q]:
//  C < Kc        - too few ads reached the threshold: status NeedLower (revise and rescan)
//  C > capacity  - overflow: the threshold becomes the Kc-th largest stored key (it strictly
//                  rises, since keys are distinct) and the query is rescanned
//  otherwise     - output mode: the first K after a sort are the result (ids, FP32 scores);
//                  prep mode: the Kc best (by radix select, in no particular order) go to the
//                  rescore scratch (id and the cross-term value carried with the candidate),
//                  with the Kc-th approximate score for the recall certificate.
__global__ __launch_bounds__(1024) void k_finalize(FinalArgs a) {
    __shared__ unsigned long long s[kCandCap];
    __shared__ uint32_t s_hist[256];
    __shared__ unsigned long long s_pref;
    __shared__ int s_rank;
    __shared__ uint32_t s_slot;
    const int q = (int)blockIdx.x;
    const int tid = (int)threadIdx.x;
    if (a.gate && *a.gate == 0u) return;
    if (a.ctl && a.ctl->error) return;
    if (!a.active[q]) return;
    const int Kc = a.kcnt[q];
    const uint32_t c = a.cand_cnt[q];
    if ((int64_t)c < (int64_t)Kc) {
        if (tid == 0) { a.status[q] = kStatusNeedLower; atomicAdd(a.unresolved, 1u); }
        return;
    }
    const int n = (int)min(c, (uint32_t)a.cap);
    const unsigned long long* src = a.cand + (int64_t)q * a.cap;
    int done = kStatusDone;
    if (a.prep || c > (uint32_t)a.cap) {
        // only the Kc-th best key is needed (a threshold; the prep pass's candidates in any
        // order): a radix select instead of a sort
        for (int i = tid; i < n; i += 1024) s[i] = src[i];
        if (tid == 0) s_slot = 0u;
        __syncthreads();
        const unsigned long long T = kth_largest(s, n, Kc, s_hist, &s_pref, &s_rank);
        if (c > (uint32_t)a.cap) {
            if (tid == 0) {
                a.thresh[2 * q] = (uint32_t)(T >> 32);
                a.thresh[2 * q + 1] = (uint32_t)T;
                a.status[q] = kStatusOverflow;
                atomicAdd(a.unresolved, 1u);
            }
            return;
        }
        // the Kc best by approximate key (the keys are distinct: exactly Kc of them reach T),
        // with their carried cross terms; the rescore sorts their exact scores
        const float* cw = a.cand_wide + (int64_t)q * a.cap;
        for (int p = tid; p < n; p += 1024) {
            const unsigned long long key = s[p];
            if (key >= T) {
                const uint32_t slot = atomicAdd(&s_slot, 1u);
                a.r_id[(int64_t)q * a.r_ld + slot] = 0xffffffffu - (uint32_t)key;
                a.r_wide[(int64_t)q * a.r_ld + slot] = cw[p];
            }
        }
        if (tid == 0) a.r_stilde[q] = key_score((uint32_t)(T >> 32));
    } else {
        int P = 64;
        while (P < n) P <<= 1;
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
        const int K = a.kq[q];
        const int64_t o = a.out_off[q];
        for (int i = tid; i < K; i += 1024) {
            const unsigned long long t = s[i];
            a.out_ids[o + i] = 0xffffffffu - (uint32_t)t;
            a.out_scores[o + i] = key_score((uint32_t)(t >> 32));
        }
        if (a.werr && !wide_precise(a.werr[q], key_score((uint32_t)(s[0] >> 32)),
                                    key_score((uint32_t)(s[K - 1] >> 32))))
            done = kStatusImprecise;
    }
    if (tid == 0) {
        a.status[q] = done;
        a.active[q] = 0u;
        if (done == kStatusImprecise) atomicAdd(a.imprecise, 1u);
    }
}


// ------------------------------------------------------------------ full sort (K > 8192)

// A query whose K exceeds the candidate buffer's sort is answered by sorting all of its
// scores: ck[a] = (~score_key(deep + wide) << 32) | a, so that ascending ck is the order
// (score descending, id ascending); the sum is the scan's own score (deep + wide is one FP32
// rounding, as fma(cell, 2^-S, deep) with the exact wide term).
__global__ void k_sort_keys(const float* deep, const float* wide, int64_t n, unsigned long long* ck) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        ck[i] = ((unsigned long long)(~score_key(deep[i] + wide[i])) << 32) | (unsigned long long)(uint32_t)i;
}

// LSD radix sort of 64-bit keys, 8 bits per pass, ascending and stable: each block of
// kSortTile keys counts its digits (hist[digit * blocks + block]); an exclusive scan of hist
// gives every (digit, block) its first output slot; the scatter ranks equal digits inside the
// block in index order (wave match by ballots, then per-wave counts in LDS).
constexpr int kSortNT = 256, kSortPer = 16, kSortTile = kSortNT * kSortPer;

__global__ __launch_bounds__(kSortNT) void k_sort_hist(const unsigned long long* in, int64_t n, int shift,
                                                       uint32_t* hist, int64_t nblk) {
    __shared__ uint32_t h[256];
    const int tid = (int)threadIdx.x;
    h[tid] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int j = 0; j < kSortPer; ++j) {
        const int64_t i = base + (int64_t)j * kSortNT + tid;
        if (i < n) atomicAdd(&h[(uint32_t)(in[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * nblk + blockIdx.x] = h[tid];
}

__global__ __launch_bounds__(kSortNT) void k_sort_scatter(const unsigned long long* in, unsigned long long* out,
                                                          int64_t n, int shift, const uint32_t* offs,
                                                          int64_t nblk) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kSortNT / 64][256];
    const int tid = (int)threadIdx.x, lane = lane_id(), w = tid >> 6;
    run[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int j = 0; j < kSortPer; ++j) {
        #pragma unroll
        for (int k = 0; k < kSortNT / 64; ++k) wcnt[k][tid] = 0u;
        __syncthreads();
        const int64_t i = base + (int64_t)j * kSortNT + tid;
        const bool ok = i < n;
        const unsigned long long x = ok ? in[i] : 0ull;
        const uint32_t d = (uint32_t)(x >> shift) & 255u;
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(ok);
        #pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint64_t below = peers & ((1ull << lane) - 1ull);
        const uint32_t rank = (uint32_t)__builtin_popcountll(below);
        if (ok && below == 0ull) wcnt[w][d] = (uint32_t)__builtin_popcountll(peers);
        __syncthreads();
        if (ok) {
            uint32_t pos = run[d] + rank;
            for (int k = 0; k < w; ++k) pos += wcnt[k][d];
            out[pos] = x;
        }
        __syncthreads();
        uint32_t add = 0;
        #pragma unroll
        for (int k = 0; k < kSortNT / 64; ++k) add += wcnt[k][tid];
        run[tid] += add;
    }
}

// The first K of the sorted keys as ids and scores.
__global__ void k_sort_out(const unsigned long long* ck, int64_t k, uint32_t* ids, float* scores) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < k; i += stride) {
        const unsigned long long v = ck[i];
        ids[i] = (uint32_t)v;
        scores[i] = key_score(~(uint32_t)(v >> 32));
    }
}

// ------------------------------------------------------------------ per-query set-up

// One wavefront per query: finiteness of the user row, status / activity from K, and the
// certificate's eps for reduced-precision scans: with u the FP32 row and u^ its BF16 copy,
//   eps = |u^ - u| Eh + |u| R + g_d (|u^| Eh + |u| E) + 2^-24 |u^| Eh
//         + 2^-22 (max(|u| E, |u^| Eh) + A_q),
// where R, Eh, E are the largest row norms of (e - e^), e^ and e, g_d = 1.01 d 2^-24 bounds
// FP32 accumulation of d products, the 2^-24 term the FP8 scale product and the last term
// the FP32 additions of the cross term (|cross term| <= A_q); everything is rounded up.
__global__ __launch_bounds__(256) void k_prep(PrepArgs a) {
    const int q = (int)(blockIdx.x * 4u + (threadIdx.x >> 6));
    const int lane = lane_id();
    if (q >= a.n_queries) return;
    const float* u = a.user + (int64_t)q * a.dim;
    bool finite = true;
    double nu = 0.0, nh = 0.0, du = 0.0;
    for (int k = lane; k < a.dim; k += 64) {
        const float x = u[k];
        finite &= isfinite(x);
        const double xd = (double)x;
        const double h = (double)__uint_as_float(bf16_bits(x) << 16);
        nu += xd * xd;
        nh += h * h;
        du += (h - xd) * (h - xd);
    }
    for (int off = 32; off > 0; off >>= 1) {
        nu += __shfl_xor(nu, off, 64);
        nh += __shfl_xor(nh, off, 64);
        du += __shfl_xor(du, off, 64);
    }
    const uint64_t bad = __ballot(!finite);
    if (lane == 0) {
        if (bad) atomicOr(&a.ctl->error, 1u);
        const int K = a.kq[q];
        a.status[q] = K > 0 ? kStatusPending : kStatusDone;
        a.active[q] = K > 0 ? 1u : 0u;
        if (a.eps) {
            nu = sqrt(nu);
            nh = sqrt(nh);
            du = sqrt(du);
            const double gd = 1.01 * a.dim * 0x1p-24;
            double e = du * a.q_norm2 + nu * a.q_err2 + gd * (nh * a.q_norm2 + nu * a.e_norm2) +
                       0x1p-24 * nh * a.q_norm2 + 0x1p-22 * (fmax(nu * a.e_norm2, nh * a.q_norm2) + a.aq[q]);
            e = e * 1.001 + 1e-30;
            a.eps[q] = __double2float_ru(e);
        }
    }
}

__global__ void k_round_reset(uint32_t* cand_cnt, int32_t n, const uint32_t* gate) {
    if (gate && *gate == 0u) return;
    for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < n; i += (int)(gridDim.x * blockDim.x))
        cand_cnt[i] = 0u;
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

int launch_prep(const PrepArgs& a, void* stream) {
    if (a.n_queries <= 0) return 0;
    hipLaunchKernelGGL(k_prep, dim3((unsigned)((a.n_queries + 3) / 4)), dim3(256), 0, (hipStream_t)stream, a);
    return last(hipSuccess);
}

int launch_round_reset(uint32_t* cand_cnt, int32_t n, const uint32_t* gate, void* stream) {
    if (n <= 0) return 0;
    const int blocks = (n + 255) / 256 < 64 ? (n + 255) / 256 : 64;
    hipLaunchKernelGGL(k_round_reset, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, cand_cnt, n, gate);
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

int launch_refine(const DecodeArgs& a, void* stream) {
    if (a.n_super <= 0) return 0;
    if (a.sshift < kSuperShift || a.sshift > kMaxSuperShift || (a.n_sub > 1 && a.sshift != kSuperShift))
        return (int)hipErrorInvalidValue;
    if (a.n_sub < 1 || a.n_sub > kSplitMaxGroups + 2) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_refine, dim3((unsigned)a.n_super), dim3(kRefineNT), 0, (hipStream_t)stream, a);
    return last(hipSuccess);
}

int launch_chunk_map(const DecodeArgs& a, void* stream) {
    if (a.n_ukeys <= 0 || a.total_chunks == 0) return 0;
    hipLaunchKernelGGL(k_chunk_map, dim3((unsigned)((a.n_ukeys + 3) / 4)), dim3(256), 0, (hipStream_t)stream, a);
    return last(hipSuccess);
}

int launch_decode(const DecodeArgs& a, int place, void* stream) {
    if (a.total_chunks == 0) return 0;
    if (a.chunks_per_wave < 1 || a.chunks_per_wave > 64) return (int)hipErrorInvalidValue;
    const uint32_t waves = (a.total_chunks + a.chunks_per_wave - 1) / a.chunks_per_wave;
    const unsigned blocks = (waves + 3u) / 4u;
    hipLaunchKernelGGL(k_decode, dim3(blocks), dim3(256), 0, (hipStream_t)stream, a, place);
    return last(hipSuccess);
}

int launch_decode_key(const ChunkHdr* chunks, const uint32_t* words, const float* weights,
                      uint32_t chunk0, uint32_t n_chunks, uint32_t post_base, uint32_t* ids,
                      float* w, void* stream) {
    if (n_chunks == 0) return 0;
    hipLaunchKernelGGL(k_decode_key, dim3(n_chunks), dim3(64), 0, (hipStream_t)stream, chunks,
                       words, weights, chunk0, post_base, ids, w);
    return last(hipSuccess);
}


bool score_dim_supported(int dim) {
    switch (dim) {
        case 16: case 32: case 48: case 64: case 80: case 96: case 112: case 128: return true;
        default: return false;
    }
}

int score_ranges(int n_work, int n_qgroups, int ctas) {
    int R = ctas / (n_qgroups > 0 ? n_qgroups : 1);
    if (R >= 8) R -= R % 8;
    if (R < 1) R = 1;
    if (R > n_work) R = n_work;
    return R;
}

int launch_score(const ScoreArgs& a_in, int dim, int mode, int ranges, void* stream) {
    if (a_in.n_work <= 0 || a_in.n_qgroups <= 0) return 0;
    if (ranges < 1 || (int64_t)ranges * a_in.n_qgroups > (1 << 24)) return (int)hipErrorInvalidValue;
    ScoreArgs a = a_in;
    a.n_ranges = ranges < a.n_work ? ranges : a.n_work;
    dim3 grid((unsigned)(a.n_ranges * a.n_qgroups));
    hipStream_t st = (hipStream_t)stream;
    const int dt = a.dtype;
    switch (dim) {
        case 16: launch_score_d<16>(a, mode, dt, grid, st); break;
        case 32: launch_score_d<32>(a, mode, dt, grid, st); break;
        case 48: launch_score_d<48>(a, mode, dt, grid, st); break;
        case 64: launch_score_d<64>(a, mode, dt, grid, st); break;
        case 80: launch_score_d<80>(a, mode, dt, grid, st); break;
        case 96: launch_score_d<96>(a, mode, dt, grid, st); break;
        case 112: launch_score_d<112>(a, mode, dt, grid, st); break;
        case 128: launch_score_d<128>(a, mode, dt, grid, st); break;
        default: return (int)hipErrorInvalidValue;
    }
    return last(hipSuccess);
}

int64_t sort_blocks(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

int launch_full_sort_topk(const float* deep, const float* wide, int64_t n, int64_t k,
                          unsigned long long* keys, unsigned long long* tmp, uint32_t* hist,
                          uint32_t* scan_tmp, uint32_t* ids, float* scores, void* stream) {
    if (n <= 0 || k <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    const int64_t nb = sort_blocks(n);
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_sort_keys, dim3(g), dim3(256), 0, st, deep, wide, n, keys);
    unsigned long long* a = keys;
    unsigned long long* b = tmp;
    for (int shift = 0; shift < 64; shift += 8) {
        hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)nb), dim3(kSortNT), 0, st, a, n, shift, hist, nb);
        const int rc = launch_excl_scan_u32(hist, hist, 256 * nb, scan_tmp, stream);
        if (rc) return rc;
        hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)nb), dim3(kSortNT), 0, st, a, b, n, shift, hist, nb);
        std::swap(a, b);
    }
    const unsigned go = (unsigned)std::min<int64_t>((k + 255) / 256, 65536);
    hipLaunchKernelGGL(k_sort_out, dim3(go), dim3(256), 0, st, a, k, ids, scores);
    return last(hipSuccess);
}

int launch_select(const SelectArgs& a, int n_queries, void* stream) {
    if (n_queries <= 0) return 0;
    hipLaunchKernelGGL(k_select, dim3((unsigned)n_queries), dim3(1024), 0, (hipStream_t)stream, a);
    return last(hipSuccess);
}

int launch_rescore(const RescoreArgs& a, int dim, int n_queries, void* stream) {
    if (n_queries <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    switch (dim) {
#define EBR_CASE(D) case D: launch_rescore_d<D>(a, n_queries, st); break;
        EBR_WIDTHS(EBR_CASE)
#undef EBR_CASE
        default: return (int)hipErrorInvalidValue;
    }
    return last(hipSuccess);
}

int launch_finalize(const FinalArgs& a, int n_queries, void* stream) {
    if (n_queries <= 0) return 0;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)n_queries), dim3(1024), 0, (hipStream_t)stream, a);
    return last(hipSuccess);
}

}  // namespace ebr

