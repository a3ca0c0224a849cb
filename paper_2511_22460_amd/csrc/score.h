// The fused scoring kernel (k_score) and the exact rescore (k_rescore), templated on the
// embedding width. Each width is compiled in a translation unit of its own (score_d*.hip).
#pragma once

#include <type_traits>

#include "device_util.h"

namespace ebr {

// ------------------------------------------------------------------ fused scoring

// One work-group (16 wavefronts at d <= 64) scores one 256-query group against a contiguous
// range of 32-ad tiles. The waves specialise:
//   waves 0..7  (consumers) - wave w owns query rows [32w, 32w + 32). Per tile: read, clear
//                             and convert its 32x32 block of the cross term, run the dot
//                             products on the matrix cores, add, select.
//   waves 8..15 (producers) - one tile ahead: stage the next tile's embedding block in LDS
//                             and accumulate its cross term into the other LDS buffer.
// One barrier per tile hands the double-buffered accumulators and embedding stage over.
//
// Embedding layout (FP32 copy): per 32-ad block, D/8 quads x 64 lanes x 4 floats, where
// quad i of lane l holds e[32b + (l & 31)][8i + 2j + (l >> 5)] for j = 0..3. Step s = 4i + j
// of the K loop then finds the B operand of v_mfma_f32_32x32x2_f32 (B[k][n] with
// k = l >> 5, n = l & 31) in component j of quad i.
//
// Accumulator layout of v_mfma_f32_32x32x2_f32: register r of lane l holds row
// 8 * (r >> 2) + 4 * (l >> 5) + (r & 3), column l & 31.
//
// Cross-term accumulators: int64 per (query, ad) in LDS (layout: acc_idx below).
constexpr int kProducerWaves = 8;

// Queries per group: 256 (8 consumer waves) up to d = 64, 128 (4 consumer waves) above, so
// that the U operand and the LDS buffers fit.
template <int D> struct ScoreShape {
    static constexpr int GQ = D <= 64 ? 256 : 128;
    static constexpr int CW = GQ / 32;
    static constexpr int NT = 64 * (CW + kProducerWaves);
};

// Accumulator cell of (query row q, ad offset o): rows are grouped by four so that the four
// consecutive rows one lane of the 32x32 matrix-core tile owns are adjacent (two 16-byte
// LDS reads); the ad column is XOR-swizzled by the row group so that the users of one posting
// (same ad, many rows) spread over the banks.
__device__ __forceinline__ int acc_idx(int q, int o) {
    return (((q >> 2) * kTileAds + (o ^ ((q >> 2) & 31))) << 2) | (q & 3);
}

// Rare path of the selection epilogue: append one survivor to its query's candidate buffer.
// Kept out of line so that the per-row buffer addresses are not hoisted into registers.
// The candidate's cross-term value is kept beside it when the scan is approximate, for the
// exact rescore.
__device__ __attribute__((noinline)) void append_candidate(unsigned long long* cand,
                                                           uint32_t* cand_cnt, float* cand_wide,
                                                           int cap, int q, uint32_t key,
                                                           uint32_t idk, float wide) {
    const uint32_t pos = atomicAdd(&cand_cnt[q], 1u);
    if (pos < (uint32_t)cap) {
        cand[(int64_t)q * cap + pos] = ((unsigned long long)key << 32) | (unsigned long long)idk;
        if (cand_wide) cand_wide[(int64_t)q * cap + pos] = wide;
    }
}

// Dense test hook: store one (query, ad) pair of terms (out of line, as above).
__device__ __attribute__((noinline)) void store_dense(float* deep_out, float* wide_out,
                                                      int64_t idx, float deep, float wide) {
    deep_out[idx] = deep;
    wide_out[idx] = wide;
}

// Bucket entry: x = (u0 << 13) | ((cnt - 1) << 5) | ad offset when the batch is one query
// group (the key's users are users[u0, u0 + cnt)), else (slot << 5) | ad offset; y = w' bits.
// Producer wave pw owns entries beg + pw + 8 * (lane + 64 r) of each tile; round r = 0 is
// prefetched one tile ahead.
struct ProdTile {
    uint32_t beg, end;  // the tile's bucket range
    uint2 e0;           // this lane's round-0 entry (valid if beg + pw + 8 * lane < end)
};


// Up to 64 bucket entries of one tile (one per lane) flattened into their (entry, user) pairs,
// 64 pairs per step: an exclusive scan of the entries' user counts places each entry's pairs;
// each entry writes its lane into the slot of its first pair in this wave's LDS row `mark`,
// a running maximum over the row gives every pair its entry, whose fields come from its lane.
// Each pair costs one users[] load, one 32 x 32 -> 64-bit multiply and one LDS atomic add.
struct EntryLanes {
    uint32_t cnt, pre, total;  // users of this lane's entry, pairs before it, pairs in all
    int base, o, w;            // users index of pair p is base + p; ad offset; weight
};

__device__ __forceinline__ EntryLanes entry_lanes(const ScoreArgs& a, int g, uint2 e, bool valid) {
    EntryLanes t;
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
    const uint32_t incl = wave_incl_sum(cnt);
    t.cnt = cnt;
    t.pre = incl - cnt;
    t.total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    t.base = (int)(u0 - t.pre);
    t.o = (int)(e.x & (kTileAds - 1));
    t.w = (int)e.y;
    return t;
}

// Entries (lanes) of the pairs of K consecutive steps s0 .. s0 + K - 1 (step s: pairs 64 s ..
// 64 s + 63), with one LDS row of 64 slots per step, so that the rows of all K steps are
// cleared, marked and read back in one round trip. carry is the entry of pair 64 s0 - 1 on
// entry (-1 before the first step) and of the last pair of the last step on return.
constexpr int kMarkRows = 4;
template <int K>
__device__ __forceinline__ void steps_entries(const EntryLanes& t, uint32_t s0, int* mark, int& carry,
                                              int* m) {
    static_assert(K <= kMarkRows, "one row per step");
    const int lane = lane_id();
    // LDS operations of one wave complete in the order issued: clear, mark, read back. Lanes
    // exchange values through the rows, so the compiler must neither reorder nor elide these
    // accesses (it sees them as one thread's accesses to unrelated addresses): compiler
    // barriers between them.
    #pragma unroll
    for (int k = 0; k < K; ++k) mark[k * 64 + lane] = -1;
    __asm__ __volatile__("" ::: "memory");
    if (t.cnt > 0u && t.pre >= 64u * s0 && t.pre < 64u * (s0 + K)) mark[t.pre - 64u * s0] = lane;
    __asm__ __volatile__("" ::: "memory");
    int mk[K];
    #pragma unroll
    for (int k = 0; k < K; ++k) mk[k] = mark[k * 64 + lane];
    __asm__ __volatile__("" ::: "memory");
    #pragma unroll
    for (int k = 0; k < K; ++k) mk[k] = wave_incl_max(mk[k]);
    #pragma unroll
    for (int k = 0; k < K; ++k) {
        m[k] = max(mk[k], carry);
        carry = __builtin_amdgcn_readlane(m[k], 63);
    }
}

// One (query, posting) pair: round(fl(m' * w')) into the query's cell (users hold m' bits,
// bucket entries w' bits).
__device__ __forceinline__ void pair_add(uint32_t* acc, uint2 ue, int o, int w) {
    const float p = __uint_as_float(ue.y) * __uint_as_float((uint32_t)w);
    atomicAdd(&acc[acc_idx((int)ue.x, o)], (uint32_t)__float2int_rn(p));
}

// The (query, multiplier) pairs of a one-group batch copied to LDS: an LDS-typed pointer, so
// that its loads are LDS reads (a generic pointer would make them flat loads).
typedef __attribute__((address_space(3))) const unsigned long long lds_uint2;

// users[i] from the LDS copy (LU) or from global memory
template <bool LU>
__device__ __forceinline__ uint2 user_at(const ScoreArgs& a, lds_uint2* lds_users, uint32_t i) {
    if constexpr (LU) {
        const unsigned long long v = lds_users[i];
        return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
    } else {
        return reinterpret_cast<const uint2*>(a.users)[i];
    }
}

// Pairs of steps [s_begin, end) of a set of entries, four steps mapped before their loads.
template <bool LU>
__device__ __forceinline__ void cross_steps(const ScoreArgs& a, const EntryLanes& t, uint32_t s_begin,
                                            int* mark, uint32_t* acc, lds_uint2* lds_users) {
    const int lane = lane_id();
    // entry of pair 64 s_begin - 1: the last lane with a non-empty entry starting before it
    int carry = -1;
    if (s_begin > 0) {
        const uint64_t before = __ballot(t.cnt > 0u && t.pre < 64u * s_begin);
        carry = before ? 63 - (int)__builtin_clzll(before) : -1;
    }
    constexpr int kSteps = kMarkRows;
    for (uint32_t s = s_begin; 64u * s < t.total; s += kSteps) {
        int m[kSteps], ub[kSteps], uo[kSteps], uw[kSteps];
        steps_entries<kSteps>(t, s, mark, carry, m);
        #pragma unroll
        for (int k = 0; k < kSteps; ++k) {
            ub[k] = __shfl(t.base, m[k], 64);
            uo[k] = __shfl(t.o, m[k], 64);
            uw[k] = __shfl(t.w, m[k], 64);
        }
        uint2 ue[kSteps];
        #pragma unroll
        for (int k = 0; k < kSteps; ++k) {
            const uint32_t p = 64u * (s + k) + (uint32_t)lane;
            if (p < t.total) ue[k] = user_at<LU>(a, lds_users, (uint32_t)ub[k] + p);
        }
        #pragma unroll
        for (int k = 0; k < kSteps; ++k)
            if (64u * (s + k) + (uint32_t)lane < t.total) pair_add(acc, ue[k], uo[k], uw[k]);
    }
}

// The first kAheadSteps steps of a tile's round-0 entries, mapped and their users[] loads
// issued one tile before the adds (the loads' latency then hides behind a whole tile).
constexpr int kAheadSteps = 6;
// (query, multiplier) pairs of one query group that are copied to LDS when they fit.
constexpr int kUsersLds = 8192;
struct PairsAhead {
    uint2 ue[kAheadSteps];
    int uo[kAheadSteps], uw[kAheadSteps];
    uint32_t total;
};

template <bool LU>
__device__ __forceinline__ PairsAhead pairs_ahead(const ScoreArgs& a, int g, uint2 e, bool valid,
                                                  int* mark, lds_uint2* lds_users) {
    const int lane = lane_id();
    const EntryLanes t = entry_lanes(a, g, e, valid);
    PairsAhead pa;
    pa.total = t.total;
    int carry = -1;
    int m[kAheadSteps] = {};
    static_assert(kMarkRows == 4 && kAheadSteps > kMarkRows && kAheadSteps <= 2 * kMarkRows,
                  "two groups of steps");
    // as many rows as the tile's pairs need (small batches have a few pairs per tile)
    if (t.total > 128u) steps_entries<4>(t, 0, mark, carry, m);
    else if (t.total > 64u) steps_entries<2>(t, 0, mark, carry, m);
    else if (t.total > 0u) steps_entries<1>(t, 0, mark, carry, m);
    if (t.total > 64u * kMarkRows) steps_entries<kAheadSteps - kMarkRows>(t, kMarkRows, mark, carry, m + kMarkRows);
    #pragma unroll
    for (int k = 0; k < kAheadSteps; ++k) {
        pa.uo[k] = 0;
        pa.uw[k] = 0;
        pa.ue[k] = make_uint2(0u, 0u);
        if (64u * k < t.total) {  // wave-uniform
            const int ub = __shfl(t.base, m[k], 64);
            pa.uo[k] = __shfl(t.o, m[k], 64);
            pa.uw[k] = __shfl(t.w, m[k], 64);
            const uint32_t p = 64u * k + (uint32_t)lane;
            if (p < t.total) pa.ue[k] = user_at<LU>(a, lds_users, (uint32_t)ub + p);
        }
    }
    return pa;
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

// Cross term of one tile (this wave's share): the prefetched round-0 pairs, the rest of
// round 0, then later rounds of entries.
template <bool LU>
__device__ __forceinline__ void prod_tile(const ScoreArgs& a, int g, int pw, const ProdTile& t,
                                          const PairsAhead& pa, int* mark, uint32_t* acc,
                                          lds_uint2* lds_users) {
    const int lane = lane_id();
    const uint2* bucket = reinterpret_cast<const uint2*>(a.bucket);
    constexpr uint32_t kRound = kProducerWaves * 64u;
    const uint32_t first = t.beg + (uint32_t)pw;
    if (first >= t.end) return;
    #pragma unroll
    for (int k = 0; k < kAheadSteps; ++k)
        if (64u * k + (uint32_t)lane < pa.total) pair_add(acc, pa.ue[k], pa.uo[k], pa.uw[k]);
    if (pa.total > 64u * kAheadSteps)
        cross_steps<LU>(a, entry_lanes(a, g, t.e0, first + kProducerWaves * (uint32_t)lane < t.end),
                        kAheadSteps, mark, acc, lds_users);
    for (uint32_t base = first + kRound; base < t.end; base += kRound) {
        const uint32_t ei = base + kProducerWaves * (uint32_t)lane;
        const bool ok = ei < t.end;
        const uint2 e = ok ? bucket[ei] : make_uint2(0u, 0u);
        cross_steps<LU>(a, entry_lanes(a, g, e, ok), 0, mark, acc, lds_users);
    }
}

template <bool LU>
__device__ __forceinline__ PairsAhead prod_ahead(const ScoreArgs& a, int g, int pw, const ProdTile& t,
                                                 int* mark, lds_uint2* lds_users) {
    const uint32_t first = t.beg + (uint32_t)pw;
    return pairs_ahead<LU>(a, g, t.e0, first + kProducerWaves * (uint32_t)lane_id() < t.end, mark, lds_users);
}


typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// One e4m3fn code -> the BF16 bits of the same value (exact: every e4m3 value is a BF16 value).
__device__ __forceinline__ uint32_t fp8_to_bf16_bits(uint32_t c) {
    const uint32_t sgn = (c & 0x80u) << 8, e = (c >> 3) & 15u, m = c & 7u;
    if (e != 0u) return sgn | ((e + 120u) << 7) | (m << 4);
    if (m == 0u) return sgn;
    const uint32_t p = 31u - __builtin_clz(m);  // m = 2^p (1 + f), value m 2^-9
    return sgn | ((p + 118u) << 7) | ((m - (1u << p)) << (7u - p));
}

// Eight e4m3fn codes (little-endian in v) -> eight BF16 values packed as one 16-byte operand.
__device__ __forceinline__ f32x4 fp8x8_to_bf16x8(uint2 v) {
    uint32_t w[4];
    #pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t src = i < 2 ? v.x : v.y;
        const int sh = (i & 1) * 16;
        w[i] = fp8_to_bf16_bits((src >> sh) & 0xffu) | (fp8_to_bf16_bits((src >> (sh + 8)) & 0xffu) << 16);
    }
    return f32x4{__uint_as_float(w[0]), __uint_as_float(w[1]), __uint_as_float(w[2]), __uint_as_float(w[3])};
}

// Embedding copies the scan can stream (DT): 0 = FP32 (32x32x2 layout), 1 = BF16 and
// 2 = FP8 (both in the 32x32x16 BF16 operand layout; FP8 is expanded to BF16 in LDS and its
// per-ad scale applied to the finished dot product).
template <int D, int DT> struct EmbStage {
    static constexpr int UNITS = DT == 0 ? (D / 8) * 64 : (D / 16) * 64;  // 16-byte LDS units
    static constexpr int PER = (UNITS + 64 * kProducerWaves - 1) / (64 * kProducerWaves);
};

// One work-group per (query group, contiguous range of tiles), persistent over its range;
// iteration `it` has the consumers score tile it from LDS buffers [it & 1] (and clear the
// accumulators they read) while the producers fill buffers [(it + 1) & 1] with tile it + 1
// and prefetch ahead. Every wave executes exactly 2 + n_it barriers.
//
// Work-group ids are laid out for the 8 XCDs of the chip (consecutive ids go to consecutive
// XCDs): all query groups of one tile range run on the same XCD, so the range's embedding
// blocks and bucket entries are fetched from HBM once and then served by that XCD's L2.
template <int D, int MODE, int DT>
__global__ __launch_bounds__(ScoreShape<D>::NT, 1) void k_score(ScoreArgs a) {
    constexpr int NQ = D / 8;
    constexpr int GQ = ScoreShape<D>::GQ;
    constexpr int CW = ScoreShape<D>::CW;
    constexpr int NT = ScoreShape<D>::NT;
    constexpr int kProdThreads = 64 * kProducerWaves;
    constexpr int UNITS = EmbStage<D, DT>::UNITS;
    constexpr int PER = EmbStage<D, DT>::PER;
    __shared__ __attribute__((aligned(16))) uint32_t s_acc[2][GQ * kTileAds];
    __shared__ f32x4 s_emb[2][NQ * 64];
    __shared__ float s_escale[2][kTileAds];
    __shared__ __attribute__((aligned(16))) float s_qscale[GQ];
    __shared__ __attribute__((aligned(16))) float s_thr[GQ];
    __shared__ uint32_t s_thr_hi[GQ];
    __shared__ uint32_t s_thr_lo[GQ];
    __shared__ uint32_t s_live[GQ];
    __shared__ int s_mark[kProducerWaves][kMarkRows * 64];
    __shared__ uint2 s_users[kUsersLds];

    const int tid = (int)threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const bool producer = wave >= CW;
    int g, range;
    {
        const int p = (int)blockIdx.x, R = a.n_ranges, nqg = a.n_qgroups;
        if (R % 8 == 0) {  // XCD-aware: range r lives on XCD r % 8 with all its query groups
            const int x = p & 7, sl = p >> 3;
            range = x + 8 * (sl / nqg);
            g = sl % nqg;
        } else {
            range = p % R;
            g = p / R;
        }
    }
    if (a.gate && *a.gate == 0u) return;
    if (a.ctl && a.ctl->error) return;
    const int qbase = g * GQ;
    const int B = a.n_queries;
    const int first = (int)(((int64_t)a.n_work * range) / a.n_ranges);
    const int n_it = (int)(((int64_t)a.n_work * (range + 1)) / a.n_ranges) - first;
    if (n_it <= 0) return;

    for (int i = tid; i < 2 * GQ * kTileAds; i += NT) (&s_acc[0][0])[i] = 0u;
    // one query group: its (query, multiplier) users fit in LDS when few enough
    const bool users_in_lds = a.packed && a.n_users <= (uint32_t)kUsersLds;
    lds_uint2* lu = (lds_uint2*)s_users;
    if (users_in_lds) {
        for (uint32_t i = (uint32_t)tid; i < a.n_users; i += (uint32_t)NT)
            s_users[i] = reinterpret_cast<const uint2*>(a.users)[i];
    }
    for (int i = tid; i < GQ; i += NT) {
        const int q = qbase + i;
        const bool in = q < B;
        s_qscale[i] = in ? (float)a.qinv[q] : 0.0f;  // 2^-S_q, |S_q| <= 100: exact in FP32
        if (MODE == 0) {
            const uint32_t hi = in ? a.thresh[2 * q] : 0xffffffffu;
            s_thr_hi[i] = hi;
            s_thr_lo[i] = in ? a.thresh[2 * q + 1] : 0xffffffffu;
            const bool live = in && a.active[q];
            // key 0 lies below every finite score's key: no threshold, every ad is a candidate
            s_thr[i] = live ? (hi == 0u ? -__builtin_inff() : key_score(hi)) : __builtin_nanf("");
            s_live[i] = live ? 1u : 0u;
        } else {
            s_live[i] = in ? 1u : 0u;
        }
    }
    auto tile_at = [&](int i) -> uint32_t {
        const int w = first + i;
        return MODE == 1 ? a.tile_list[w] : (uint32_t)w;  // the sample pass walks a tile list
    };
    __syncthreads();

    if (producer) {
        // the producer is instantiated for users in LDS and in global memory (uniform choice)
        auto produce = [&](auto lds_tag) {
            constexpr bool LU = decltype(lds_tag)::value;
            const int pw = wave - CW;
            const int ptid = tid - 64 * CW;
            // pipeline: bucket bounds two tiles ahead, round-0 entries one tile ahead, the
            // embedding block in registers two tiles ahead (written to LDS one tile ahead)
            struct Raw {
                f32x4 u[PER];    // FP32 / BF16 units
                uint2 c[PER];    // FP8 codes
                float scale;     // FP8: the scale of ad (ptid) of the tile
            };
            auto emb_load = [&](uint32_t t, Raw& r) {
                #pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int j = ptid + k * kProdThreads;
                    if (j < UNITS) {
                        if (DT == 2) r.c[k] = reinterpret_cast<const uint2*>(a.emb)[(int64_t)t * UNITS + j];
                        else r.u[k] = reinterpret_cast<const f32x4*>(a.emb)[(int64_t)t * UNITS + j];
                    }
                }
                if (DT == 2 && ptid < kTileAds) r.scale = a.fp8_scale[(int64_t)t * kTileAds + ptid];
            };
            auto emb_store = [&](int buf, const Raw& r) {
                #pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int j = ptid + k * kProdThreads;
                    if (UNITS % kProdThreads == 0 || j < UNITS)
                        s_emb[buf][j] = DT == 2 ? fp8x8_to_bf16x8(r.c[k]) : r.u[k];
                }
                if (DT == 2 && ptid < kTileAds) s_escale[buf][ptid] = r.scale;
            };
            const uint32_t t0 = tile_at(0);
            {
                Raw e0;
                emb_load(t0, e0);
                emb_store(0, e0);
                const ProdTile p0 = prod_entries(a, prod_bounds(a, t0), pw);
                prod_tile<LU>(a, g, pw, p0, prod_ahead<LU>(a, g, pw, p0, s_mark[pw], lu), s_mark[pw], s_acc[0], lu);
            }
            // Tiles u = 1 .. n_it - 1 are filled in iteration u - 1. Every load is issued two
            // iterations before its first use, so the state is kept in two sets, for odd and even
            // u. Before the step for tile u its set holds: the embedding block of u (loaded), the
            // first pairs of u (loaded), the entries of u and of u + 2, the bounds of u + 4.
            struct Set {
                Raw e;
                PairsAhead pa;
                ProdTile pc, pn;
                uint2 bn;
            };
            Set so{}, se{};
            auto entries_of = [&](int u) { return prod_entries(a, prod_bounds(a, tile_at(u)), pw); };
            auto fill = [&](Set& st, int u) {  // prologue: the state before the step for tile u
                if (u >= n_it) return;
                emb_load(tile_at(u), st.e);
                st.pc = entries_of(u);
                st.pa = prod_ahead<LU>(a, g, pw, st.pc, s_mark[pw], lu);
                if (u + 2 < n_it) st.pn = entries_of(u + 2);
                if (u + 4 < n_it) st.bn = prod_bounds(a, tile_at(u + 4));
            };
            fill(so, 1);
            fill(se, 2);
            __syncthreads();
            auto step = [&](int u, Set& st) {
                const int nb = u & 1;  // buffer of tile u (the consumers read it in iteration u)
                emb_store(nb, st.e);
                if (u + 2 < n_it) emb_load(tile_at(u + 2), st.e);
                prod_tile<LU>(a, g, pw, st.pc, st.pa, s_mark[pw], s_acc[nb], lu);
                if (u + 2 < n_it) {
                    st.pa = prod_ahead<LU>(a, g, pw, st.pn, s_mark[pw], lu);
                    st.pc = st.pn;
                }
                if (u + 4 < n_it) st.pn = prod_entries(a, st.bn, pw);
                if (u + 6 < n_it) st.bn = prod_bounds(a, tile_at(u + 6));
                __syncthreads();
            };
            for (int u = 1; u < n_it; u += 2) {
                step(u, so);
                if (u + 1 < n_it) step(u + 1, se);
            }
            __syncthreads();  // the consumers' last iteration
        };
        if (users_in_lds) produce(std::true_type{});
        else produce(std::false_type{});
        return;
    }

    // consumer, groups of at most 2 CW queries (FP32, d <= 64): lane (wave w, half h) owns the
    // cell of row 2 w + h and ad column lane mod 32 and computes its dot product as a chain of
    // FMAs in the order and rounding of the 32x32x2 matrix product (per step the even
    // dimension, then the odd one, each rounded), so its scores are bit-identical to the
    // matrix-core path's, while the work is spread over all consumer waves instead of a
    // 32-row product on one SIMD for a handful of rows.
    if (DT == 0 && MODE != 2 && D <= 64 && B - qbase <= 2 * CW) {
        const int o = lane & 31;
        const int row = 2 * wave + (lane >> 5);
        const int q = qbase + row;
        const bool qok = q < B;
        const bool wave_on = qbase + 2 * wave < B;  // wave-uniform
        float us[D];
#pragma unroll
        for (int d = 0; d < D; ++d) us[d] = qok ? a.user[(int64_t)q * D + d] : 0.0f;
        __syncthreads();
        for (int it = 0; it < n_it; ++it) {
            if (wave_on) {
                const int cur = it & 1;
                uint32_t* acc = s_acc[cur];
                const f32x4* eb = s_emb[cur];
                float deep = 0.0f;
#pragma unroll
                for (int i = 0; i < NQ; ++i) {
                    const f32x4 e0 = eb[i * 64 + o];       // dimensions 8 i + 2 j
                    const f32x4 e1 = eb[i * 64 + 32 + o];  // dimensions 8 i + 2 j + 1
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        deep = fmaf(us[8 * i + 2 * j], e0[j], deep);
                        deep = fmaf(us[8 * i + 2 * j + 1], e1[j], deep);
                    }
                }
                const int cell = acc_idx(row, o);
                const uint32_t wv = acc[cell];
                acc[cell] = 0u;
                const float sq = s_qscale[row];
                const float sc = fmaf((float)(int)wv, sq, deep);
                const int64_t ad = (int64_t)tile_at(it) * kTileAds + o;
                const bool ad_ok = ad < a.n_ads;
                if (MODE == 1) {
                    if (qok)
                        a.sample_keys[(int64_t)q * a.sample_ld + (uint32_t)(first + it) * kTileAds + (uint32_t)o] =
                            ad_ok ? score_key(sc) : 0u;
                } else {
                    const bool pass = qok && ad_ok && sc >= s_thr[row];  // NaN threshold: never
                    if (__ballot(pass) != 0ull && pass) {
                        const uint32_t idk = 0xffffffffu - (uint32_t)ad;
                        const uint32_t key = score_key(sc);
                        if (key > s_thr_hi[row] || (key == s_thr_hi[row] && idk >= s_thr_lo[row]))
                            append_candidate(a.cand, a.cand_cnt, a.cand_wide, a.cap, q, key, idk,
                                             (float)(int)wv * sq);
                    }
                }
            }
            __syncthreads();
        }
        return;
    }

    // consumer: A operand (user rows) of this wave's 32-query block, kept in registers:
    // FP32 pairs for the 32x32x2 FP32 product, or BF16 octets (round to nearest even)
    const int q0 = qbase + wave * 32;
    constexpr int NUR = DT == 0 ? D / 2 : 1;
    constexpr int NUB = DT == 0 ? 1 : D / 16;
    float ureg[NUR];
    bf16x8 ubf[NUB];
    {
        const int q = q0 + (lane & 31);
        if (DT == 0) {
            const int kofs = lane >> 5;
            #pragma unroll
            for (int s = 0; s < NUR; ++s)
                ureg[s] = (q < B) ? a.user[(int64_t)q * D + 2 * s + kofs] : 0.0f;
        } else {
            const int kofs = 8 * (lane >> 5);
            #pragma unroll
            for (int s = 0; s < NUB; ++s) {
                uint32_t w[4];
                #pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float x0 = (q < B) ? a.user[(int64_t)q * D + 16 * s + kofs + 2 * i] : 0.0f;
                    const float x1 = (q < B) ? a.user[(int64_t)q * D + 16 * s + kofs + 2 * i + 1] : 0.0f;
                    w[i] = bf16_bits(x0) | (bf16_bits(x1) << 16);
                }
                ubf[s] = __builtin_bit_cast(bf16x8, f32x4{__uint_as_float(w[0]), __uint_as_float(w[1]),
                                                          __uint_as_float(w[2]), __uint_as_float(w[3])});
            }
        }
    }
    bool wave_live = false;
    if (q0 < B) {
        uint32_t any = 0;
        for (int i = 0; i < 32; ++i) any |= s_live[wave * 32 + i];
        wave_live = any != 0;
    }
    __syncthreads();

    // this lane's rows: group g4 (0..3) holds rows rg(g4) .. rg(g4) + 3 of the group's 256
    auto rg = [&](int g4) { return wave * 32 + 8 * g4 + 4 * (lane >> 5); };
    const int o = lane & 31;
    for (int it = 0; it < n_it; ++it) {
        const int cur = it & 1;
        uint32_t* acc = s_acc[cur];
        if (!wave_live) {
            // rows of queries in the batch but inactive in this round still receive cross
            // terms: keep the buffer clear for its next use. Rows past the batch are never
            // written (the buffers start cleared), so their waves only keep the barrier count.
            if (q0 < B) {
                #pragma unroll
                for (int g4 = 0; g4 < 4; ++g4)
                    *reinterpret_cast<uint4*>(acc + acc_idx(rg(g4), o)) = make_uint4(0u, 0u, 0u, 0u);
            }
            __syncthreads();
            continue;
        }
        // products first: the tile's B operands are read from LDS up to eight quads ahead of
        // the products that use them, so one LDS latency is exposed per tile
        const uint32_t tile = tile_at(it);
        f32x16 c = {};
        const f32x4* eb = s_emb[cur];
        if (DT == 0) {
            constexpr int W = NQ < 8 ? NQ : 8;
            f32x4 ev[W];
            #pragma unroll
            for (int i = 0; i < W; ++i) ev[i] = eb[i * 64 + lane];
            #pragma unroll
            for (int i = 0; i < NQ; ++i) {
                const f32x4 e4 = ev[i % W];
                if (i + W < NQ) ev[i % W] = eb[(i + W) * 64 + lane];
                #pragma unroll
                for (int j = 0; j < 4; ++j)
                    c = __builtin_amdgcn_mfma_f32_32x32x2f32(ureg[4 * i + j], e4[j], c, 0, 0, 0);
            }
        } else {
            bf16x8 ev[NUB];
            #pragma unroll
            for (int s2 = 0; s2 < NUB; ++s2) ev[s2] = __builtin_bit_cast(bf16x8, eb[s2 * 64 + lane]);
            #pragma unroll
            for (int s2 = 0; s2 < NUB; ++s2)
                c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ubf[s2], ev[s2], c, 0, 0, 0);
        }
        // then the cross term of this lane's 16 cells: read (all reads in flight together),
        // cleared for the buffer's next use, converted to FP32
        float wd[16];
        {
            uint4 av[4];
            #pragma unroll
            for (int g4 = 0; g4 < 4; ++g4) av[g4] = *reinterpret_cast<const uint4*>(acc + acc_idx(rg(g4), o));
            #pragma unroll
            for (int g4 = 0; g4 < 4; ++g4)
                *reinterpret_cast<uint4*>(acc + acc_idx(rg(g4), o)) = make_uint4(0u, 0u, 0u, 0u);
            #pragma unroll
            for (int g4 = 0; g4 < 4; ++g4) {
                wd[4 * g4] = (float)(int)av[g4].x;  // the row's scale is applied below
                wd[4 * g4 + 1] = (float)(int)av[g4].y;
                wd[4 * g4 + 2] = (float)(int)av[g4].z;
                wd[4 * g4 + 3] = (float)(int)av[g4].w;
            }
        }
        const float escale = DT == 2 ? s_escale[cur][o] : 1.0f;
        const int64_t ad = (int64_t)tile * kTileAds + o;
        const bool ad_ok = ad < a.n_ads;
        float sc[16];
        bool pass = false;
        // sample pass: row base of this wave's block plus a 32-bit offset per row
        uint32_t* skeys = MODE == 1 ? a.sample_keys + (int64_t)q0 * a.sample_ld : nullptr;
        const uint32_t scol = (uint32_t)(first + it) * kTileAds + (uint32_t)o;
        #pragma unroll
        for (int g4 = 0; g4 < 4; ++g4) {
            const int r0 = rg(g4);
            const f32x4 th = *reinterpret_cast<const f32x4*>(s_thr + r0);
            const f32x4 sq = *reinterpret_cast<const f32x4*>(s_qscale + r0);
            #pragma unroll
            for (int k = 0; k < 4; ++k) {
                // the cross term's integer sum times 2^-S_q (exact); the score is one fused
                // multiply-add, the same value as the sum deep + wide
                const float wide = wd[4 * g4 + k] * sq[k];
                const float deep = DT == 2 ? c[4 * g4 + k] * escale : c[4 * g4 + k];
                if (MODE == 2) {
                    const int q = qbase + r0 + k;
                    if (ad_ok && q < B)
                        store_dense(a.deep_out, a.wide_out, (int64_t)q * a.n_ads + ad, deep, wide);
                } else if (MODE == 1) {
                    const int rl = r0 - wave * 32 + k;
                    if (q0 + rl < B)
                        skeys[(uint32_t)rl * (uint32_t)a.sample_ld + scol] = ad_ok ? score_key(fmaf(wd[4 * g4 + k], sq[k], deep)) : 0u;
                } else {
                    sc[4 * g4 + k] = fmaf(wd[4 * g4 + k], sq[k], deep);
                    pass |= sc[4 * g4 + k] >= th[k];  // NaN threshold: never
                }
            }
        }
        if (MODE == 0 && __ballot(pass && ad_ok) != 0ull) {
            // rare: exact (key, id) comparison against the threshold, then append
            if (pass && ad_ok) {
                const uint32_t idk = 0xffffffffu - (uint32_t)ad;
                #pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int ql = wave * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    if (sc[r] >= s_thr[ql]) {
                        const uint32_t key = score_key(sc[r]);
                        if (key > s_thr_hi[ql] || (key == s_thr_hi[ql] && idk >= s_thr_lo[ql]))
                            append_candidate(a.cand, a.cand_cnt, a.cand_wide, a.cap, qbase + ql, key, idk,
                                             wd[r] * s_qscale[ql]);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Exact FP32 rescore of the Kc approximate-best candidates of query q (one work-group): each
// candidate's FP32 row is gathered from the 32x32x2 layout by one thread, whose dot product is
// the FP32 scan's own FMA chain, so the rescored score is bit-identical to the FP32 scan's;
// the score adds the carried cross term. The Kc exact keys are sorted and the first K
// written. Certificate:
// every ad outside the candidates has an approximate score <= the Kc-th approximate score s~
// and differs from its exact score by at most eps_q, so s~ + eps_q < (K-th exact score)
// proves the result is the exact top-K; otherwise the query is marked uncertified.
template <int D>
__global__ __launch_bounds__(1024) void k_rescore(RescoreArgs a) {
    constexpr int NQ = D / 8;
    __shared__ unsigned long long s[kMaxK];
    __shared__ float s_u[D];
    const int q = (int)blockIdx.x;
    const int tid = (int)threadIdx.x;
    const int K = a.kq[q];
    if (a.ctl && a.ctl->error) return;
    if (a.skip && *a.skip != 0u) return;
    if (K <= 0 || a.status[q] != kStatusDone) return;
    const int Kc = a.kcnt[q];
    for (int i = tid; i < D; i += 1024) s_u[i] = a.user[(int64_t)q * D + i];
    __syncthreads();
    // one thread per candidate: the dot product is one FMA chain over the dimensions in
    // order, which is what the FP32 scan's 32x32x2 products compute (the k = 0 dimension of
    // each step, then the k = 1 one, each rounded), so a rescored score has the FP32 scan's
    // bits; the cross term is the scan's exact value.
    const f32x4* emb = reinterpret_cast<const f32x4*>(a.emb);
    for (int r = tid; r < Kc; r += 1024) {
        const uint32_t id = a.r_id[(int64_t)q * a.r_ld + r];
        const int64_t b = id >> kTileShift;
        const int o = (int)(id & (kTileAds - 1));
        f32x4 e0[NQ], e1[NQ];
        #pragma unroll
        for (int i = 0; i < NQ; ++i) {
            e0[i] = emb[(b * NQ + i) * 64 + o];       // dimensions 8 i + 2 j
            e1[i] = emb[(b * NQ + i) * 64 + 32 + o];  // dimensions 8 i + 2 j + 1
        }
        float deep = 0.0f;
        #pragma unroll
        for (int i = 0; i < NQ; ++i) {
            #pragma unroll
            for (int j = 0; j < 4; ++j) {
                deep = fmaf(s_u[8 * i + 2 * j], e0[i][j], deep);
                deep = fmaf(s_u[8 * i + 2 * j + 1], e1[i][j], deep);
            }
        }
        const float sc = deep + a.r_wide[(int64_t)q * a.r_ld + r];
        s[r] = ((unsigned long long)score_key(sc) << 32) | (unsigned long long)(0xffffffffu - id);
    }
    int P = 64;
    while (P < Kc) P <<= 1;
    for (int i = Kc + tid; i < P; i += 1024) s[i] = 0ull;
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
    const int64_t o = a.out_off[q];
    for (int i = tid; i < K; i += 1024) {
        const unsigned long long t = s[i];
        a.out_ids[o + i] = 0xffffffffu - (uint32_t)t;
        a.out_scores[o + i] = key_score((uint32_t)(t >> 32));
    }
    if (tid == 0) {
        bool cert = (int64_t)Kc >= a.n_ads;
        if (!cert) {
            const double sk = (double)key_score((uint32_t)(s[K - 1] >> 32));
            cert = (double)a.r_stilde[q] + (double)a.eps[q] < sk;
        }
        if (!cert) {
            a.status[q] = kStatusUncertified;
            atomicAdd(a.uncertified, 1u);
        }
    }
}

template <int D, int DT>
static void launch_score_dt(const ScoreArgs& a, int mode, dim3 grid, hipStream_t st) {
    constexpr int NT = ScoreShape<D>::NT;
    if (mode == 0) hipLaunchKernelGGL((k_score<D, 0, DT>), grid, dim3(NT), 0, st, a);
    else if (mode == 1) hipLaunchKernelGGL((k_score<D, 1, DT>), grid, dim3(NT), 0, st, a);
    else hipLaunchKernelGGL((k_score<D, 2, DT>), grid, dim3(NT), 0, st, a);
}

template <int D>
void launch_score_d(const ScoreArgs& a, int mode, int dt, dim3 grid, hipStream_t st) {
    if (dt == 0) launch_score_dt<D, 0>(a, mode, grid, st);
    else if (dt == 1) launch_score_dt<D, 1>(a, mode, grid, st);
    else launch_score_dt<D, 2>(a, mode, grid, st);
}

template <int D>
void launch_rescore_d(const RescoreArgs& a, int n_queries, hipStream_t st) {
    hipLaunchKernelGGL(k_rescore<D>, dim3((unsigned)n_queries), dim3(1024), 0, st, a);
}

}  // namespace ebr
