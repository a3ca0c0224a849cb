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
// Embedding layout (FP32 copy): row-major, the rows padded to a multiple of 32 (so that an
// ad's row is 2 x 128-byte lines when it is gathered on its own). The stager writes a tile's
// 16-byte chunk c (dimensions 4c .. 4c + 3) of ad o to LDS quad i = c >> 1, lane
// ((c & 1) << 5 | o) XOR 2i (the XOR spreads the stager's writes over the banks), so that step
// s = 4i + j of the K loop finds the B operand of v_mfma_f32_32x32x2_f32 (B[k][n] with
// k = l >> 5, n = l & 31) in component j of that quad: dimension 8i + 4k + j. The user rows
// (A operand) take the same dimension order.
//
// Accumulator layout of v_mfma_f32_32x32x2_f32: register r of lane l holds row
// 8 * (r >> 2) + 4 * (l >> 5) + (r & 3), column l & 31.
//
// Cross-term accumulators: one fixed-point cell per (query, ad) in LDS (layout: acc_idx
// below), 32-bit, or 64-bit (W64) for queries whose 32-bit quantum is too coarse.
constexpr int kProducerWaves = 8;
// Producer waves: one stager (embedding blocks into LDS), the others accumulate the cross term.
constexpr int kStageWaves = 1;
constexpr int kCrossWaves = kProducerWaves - kStageWaves;
constexpr int kStageThreads = 64 * kStageWaves;

// Candidate ring: entries per consumer wave and ring half (the mean is below one per tile at
// the top-K sizes served; a full slice falls back to a direct append).
constexpr int kRingSlice = 8;

template <bool W64> using AccT = typename std::conditional<W64, unsigned long long, uint32_t>::type;

// Queries per group: 256 (8 consumer waves) up to d = 64 with 32-bit cells, else 128 (4
// consumer waves), so that the U operand and the LDS buffers fit.
template <int D, bool W64 = false> struct ScoreShape {
    static constexpr int GQ = score_gq(D, W64);
    static constexpr int CW = GQ / 32;
    static constexpr int NT = 64 * (CW + kProducerWaves);
    // (query, multiplier) records in LDS: a one-group batch's (when they fit), or a group's
    // users of the hot keys of split buckets
    static constexpr int USERS_LDS = score_users_lds(D, W64);
};

// FP32 -> int64, round to nearest even; |p| <= 2^62 (the planner's bound for 64-bit cells).
// The integer value rint(p) is split exactly into 32-bit halves of its magnitude.
__device__ __forceinline__ long long f32_to_i64_rn(float p) {
    const float r = rintf(p);
    const float m = fabsf(r);
    const float hi = floorf(m * 0x1p-32f);   // <= 2^30
    const float lo = fmaf(hi, -0x1p32f, m);  // m - hi 2^32: exact, in [0, 2^32)
    const unsigned long long v =
        ((unsigned long long)(uint32_t)hi << 32) | (unsigned long long)(uint32_t)lo;
    return r < 0.0f ? -(long long)v : (long long)v;
}

// A cell's fixed-point sum as FP32 (one rounding, to nearest even).
__device__ __forceinline__ float acc_value(uint32_t v) { return (float)(int)v; }
__device__ __forceinline__ float acc_value(unsigned long long v) { return (float)(long long)v; }

// Four consecutive cells (one lane's rows r .. r + 3 of a column): read, and clear.
__device__ __forceinline__ void read4(const uint32_t* p, uint32_t* v) {
    const uint4 x = *reinterpret_cast<const uint4*>(p);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}
__device__ __forceinline__ void read4(const unsigned long long* p, unsigned long long* v) {
    const ulonglong2 x = reinterpret_cast<const ulonglong2*>(p)[0];
    const ulonglong2 y = reinterpret_cast<const ulonglong2*>(p)[1];
    v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
}
__device__ __forceinline__ void clear4(uint32_t* p) {
    *reinterpret_cast<uint4*>(p) = make_uint4(0u, 0u, 0u, 0u);
}
__device__ __forceinline__ void clear4(unsigned long long* p) {
    reinterpret_cast<ulonglong2*>(p)[0] = make_ulonglong2(0ull, 0ull);
    reinterpret_cast<ulonglong2*>(p)[1] = make_ulonglong2(0ull, 0ull);
}

// Accumulator cell of (query row q, ad offset o): rows are grouped by four so that the four
// consecutive rows one lane of the 32x32 matrix-core tile owns are adjacent (two 16-byte
// LDS reads); the ad column is XOR-swizzled by the row group so that the users of one posting
// (same ad, many rows) spread over the banks.
__host__ __device__ constexpr int acc_idx(int q, int o) {
    return (((q >> 2) * kTileAds + (o ^ ((q >> 2) & 31))) << 2) | (q & 3);
}

// the user records' cell codes (acc_row_code) address the same cells as acc_idx
constexpr bool acc_codes_match() {
    for (int w = 0; w < 2; ++w)
        for (int q = 0; q < 256; ++q)
            for (int o = 0; o < kTileAds; ++o) {
                const uint32_t c = acc_row_code((uint32_t)q, w == 1);
                const uint32_t byte = (c & 0xffffu) + (((uint32_t)o << (w ? 5 : 4)) ^ (c >> 16));
                if (byte != (uint32_t)acc_idx(q, o) * (w ? 8u : 4u)) return false;
            }
    return true;
}
static_assert(acc_codes_match(), "cell codes and acc_idx disagree");

// (key, id) at or above the threshold (hi, lo), in the order of the selection keys. Evaluated
// without short-circuit branches: with them, a value selected after the branches (the id of a
// candidate whose key ties the threshold) was found cleared in the compiled code.
__device__ __forceinline__ bool key_passes(uint32_t key, uint32_t idk, uint32_t hi, uint32_t lo) {
    return (key > hi) | ((key == hi) & (idk >= lo));
}

// Append one survivor to its query's candidate buffer (rare path of the selection epilogue).
// The empty asm statement hides q's value from the optimizer, so that the per-row buffer
// addresses of an unrolled row loop are computed here and not hoisted into registers (a call
// would do the same, but makes the caller save its registers). The candidate's cross-term
// value is kept beside it when the scan is approximate, for the exact rescore.
__device__ __forceinline__ void append_candidate(unsigned long long* cand, uint32_t* cand_cnt, float* cand_wide,
                                                 int cap, int q, uint32_t key, uint32_t idk, float wide) {
    __asm__ volatile("" : "+v"(q));
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
// With split buckets a tile's shared entries are [beg, mid) of hot keys (users in the LDS
// table) and [mid, end) of warm keys (users through users_off); a group's cold pairs are
// added by the stager wave. Cross-term wave xw owns entries beg + xw + kCrossWaves * (lane +
// 64 r) of each tile; round r = 0 is prefetched one tile ahead.
struct Bounds {
    uint32_t beg, mid, end;
};

struct ProdTile {
    Bounds b;
    uint2 e0;  // this lane's round-0 entry
};

// Users one lane adds per item: an item is (bucket entry, up to kUserChunk of the users of the
// entry's key), so a lane runs kUserChunk independent (load, multiply, LDS add) sequences per
// item and the cost of assigning items to lanes is shared by that many pairs. An entry with
// cnt users has nch = ceil(cnt / kUserChunk) items; item c takes the users c + j nch
// (j < kUserChunk, below cnt), so that the lanes holding an entry's consecutive items read
// consecutive users (one LDS bank each) at every j. Four: every slot of an item adds (an
// unused one adds 0), and most keys have few users in a batch; measured against eight, a
// single query's scan 0.99 -> 0.84 ms, 16 queries 1.41 -> 1.18, 256 BF16 2.42 -> 2.35, FP32
// unchanged.
constexpr int kUserChunk = 4;

// The (query, multiplier) records and the hot-key table in LDS: LDS-typed pointers, so that
// their loads are LDS reads (a generic pointer would make them flat loads).
typedef __attribute__((address_space(3))) const unsigned long long lds_uint2;
typedef __attribute__((address_space(3))) const uint32_t lds_u32;

// Where an entry's (query, multiplier) records are: 0 = users[] in global memory, 1 = the LDS
// records, 2 = per entry (split buckets: hot keys in LDS, warm keys in global memory).
constexpr int kSrcGlobal = 0, kSrcLds = 1, kSrcMixed = 2;
constexpr uint32_t kCoLds = 1u << 14;  // EntryItems::co: this entry's records are in LDS

// Up to 64 bucket entries of one tile (one per lane) cut into items and laid out 64 items per
// step: an exclusive scan of the entries' item counts places each entry's items; each entry
// writes (first item << 6 | lane) into the slot of its first item in this wave's LDS row
// `mark`, and a running maximum over the row gives every item its entry and, from the high
// bits, its chunk within the entry.
struct EntryItems {
    uint32_t nch, pre, total;  // items of this lane's entry, items before it, items in all
    uint32_t u0;               // users index of the entry's first user
    uint32_t co;               // (users count << 5) | ad offset, kCoLds if the users are in LDS
    uint32_t w;                // w' bits
};

template <int SRC>
__device__ __forceinline__ EntryItems entry_items(const ScoreArgs& a, int g, uint2 e, bool valid, bool hot,
                                                  lds_u32* s_hot) {
    EntryItems t;
    uint32_t cnt = 0, u0 = 0, lds = SRC == kSrcLds ? kCoLds : 0u;
    if (a.packed) {  // wave-uniform; no loads
        u0 = valid ? e.x >> 13 : 0u;
        cnt = valid ? ((e.x >> kTileShift) & 255u) + 1u : 0u;
    } else {
        // Loads are issued by every lane (lanes without a record read index 0) and their
        // values selected, so that no load sits in a branch: the compiler then knows how many
        // loads are in flight at each wait and leaves the prefetched ones outstanding.
        const bool hl = SRC == kSrcMixed && valid && hot;
        const bool gl = valid && !hl;
        const uint32_t slot = gl ? (e.x >> kTileShift) * (uint32_t)a.n_qgroups + (uint32_t)g : 0u;
        const uint32_t o0 = a.users_off[slot], o1 = a.users_off[slot + 1];
        if (SRC == kSrcMixed) {
            const uint32_t h = s_hot[hl ? e.x >> kTileShift : 0u];
            u0 = hl ? h >> 9 : (gl ? o0 : 0u);
            cnt = hl ? h & 511u : (gl ? o1 - o0 : 0u);
            lds = hl ? kCoLds : 0u;
        } else {
            u0 = gl ? o0 : 0u;
            cnt = gl ? o1 - o0 : 0u;
        }
    }
    t.nch = (cnt + (kUserChunk - 1)) / kUserChunk;
    const uint32_t incl = wave_incl_sum(t.nch);
    t.pre = incl - t.nch;
    t.total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    t.u0 = u0;
    t.co = (cnt << kTileShift) | (e.x & (kTileAds - 1)) | lds;
    t.w = e.y;
    return t;
}

// Owner of item 64 s + lane: (first item of the owning entry << 6) | its lane, or -1 past the
// items. carry is the owner of item 64 s - 1 on entry (-1 before the first step) and of item
// 64 s + 63 on return.
__device__ __forceinline__ int step_owner(const EntryItems& t, uint32_t s, int* mark, int& carry) {
    const int lane = lane_id();
    // LDS operations of one wave complete in the order issued: clear, mark, read back. Lanes
    // exchange values through the row, so the compiler must neither reorder nor elide these
    // accesses (it sees them as one thread's accesses to unrelated addresses): compiler
    // barriers between them.
    mark[lane] = -1;
    __asm__ __volatile__("" ::: "memory");
    if (t.nch > 0u && t.pre >= 64u * s && t.pre < 64u * (s + 1))
        mark[t.pre - 64u * s] = (int)((t.pre << 6) | (uint32_t)lane);
    __asm__ __volatile__("" ::: "memory");
    int mk = mark[lane];
    __asm__ __volatile__("" ::: "memory");
    const int m = max(wave_incl_max(mk), carry);
    carry = __builtin_amdgcn_readlane(m, 63);
    return m;
}

// owner of item 64 s_begin - 1: the last lane with items whose first item lies before it
__device__ __forceinline__ int carry_before(const EntryItems& t, uint32_t s_begin) {
    if (s_begin == 0) return -1;
    const uint64_t before = __ballot(t.nch > 0u && t.pre < 64u * s_begin);
    if (!before) return -1;
    const int l = 63 - (int)__builtin_clzll(before);
    return __builtin_amdgcn_readlane((int)((t.pre << 6) | (uint32_t)lane_id()), l);
}

// One item mapped to this lane: its users' (query row, m') pairs loaded, the entry's ad offset
// and weight; bit j of valid: user j exists (0: no item).
struct ItemLoad {
    uint2 ue[kUserChunk];
    int o, w;
    uint32_t valid;
};

// The item's users[idx[j]] (bit j of valid) from the LDS records or from global memory;
// users outside valid read index 0 (never added). The reads are unconditional and not
// selected after the load (see entry_items), so a prefetched item's loads stay in flight. With
// split buckets a lane's users are in LDS (hot key) or in global memory (warm key); the global
// reads are issued only when some lane of the wave has a warm item, and then selected at once.
template <int SRC>
__device__ __forceinline__ void users_load(const ScoreArgs& a, lds_uint2* lds_users, const uint32_t* idx,
                                           uint32_t valid, uint32_t fl, uint2* ue) {
    const uint2* gu = reinterpret_cast<const uint2*>(a.users);
    if (SRC == kSrcGlobal) {
        #pragma unroll
        for (int j = 0; j < kUserChunk; ++j) ue[j] = gu[((valid >> j) & 1u) ? idx[j] : 0u];
        return;
    }
    const bool l = SRC == kSrcLds || (fl & kCoLds) != 0u;
    #pragma unroll
    for (int j = 0; j < kUserChunk; ++j) {
        const unsigned long long v = lds_users[((valid >> j) & 1u) && l ? idx[j] : 0u];
        ue[j] = make_uint2((uint32_t)v, (uint32_t)(v >> 32));
    }
    if (SRC == kSrcMixed && __ballot(valid != 0u && !l) != 0ull) {
        uint2 gv[kUserChunk];
        #pragma unroll
        for (int j = 0; j < kUserChunk; ++j) gv[j] = gu[((valid >> j) & 1u) && !l ? idx[j] : 0u];
        #pragma unroll
        for (int j = 0; j < kUserChunk; ++j) ue[j] = l ? ue[j] : gv[j];
    }
}

template <int SRC>
__device__ __forceinline__ ItemLoad item_load(const ScoreArgs& a, const EntryItems& t, uint32_t s, int m,
                                              lds_uint2* lds_users) {
    ItemLoad it;
    const int lane = lane_id();
    const uint32_t k = 64u * s + (uint32_t)lane;
    const int ml = m & 63;
    const uint32_t u0 = (uint32_t)__shfl((int)t.u0, ml, 64);
    const uint32_t co = (uint32_t)__shfl((int)t.co, ml, 64);
    it.w = __shfl((int)t.w, ml, 64);
    it.o = (int)(co & (kTileAds - 1));
    const uint32_t c = k - ((uint32_t)m >> 6);  // item (chunk) index within its entry
    const uint32_t cnt = (co >> kTileShift) & 511u;
    const uint32_t nch = (cnt + (kUserChunk - 1)) / kUserChunk;
    const bool on = k < t.total && m >= 0;
    const uint32_t fl = co & kCoLds;
    it.valid = 0u;
    uint32_t idx[kUserChunk];
    #pragma unroll
    for (int j = 0; j < kUserChunk; ++j) {
        const uint32_t uj = c + (uint32_t)j * nch;
        it.valid |= on && uj < cnt ? (1u << j) : 0u;
        idx[j] = u0 + uj;
    }
    users_load<SRC>(a, lds_users, idx, it.valid, fl, it.ue);
    return it;
}

// Every entry of the wave has at most kUserChunk users (one item each): the item of lane l is
// lane l's own entry, with no search.
template <int SRC>
__device__ __forceinline__ ItemLoad own_item_load(const ScoreArgs& a, const EntryItems& t, lds_uint2* lds_users) {
    ItemLoad it;
    const uint32_t cnt = (t.co >> kTileShift) & 511u;
    const uint32_t fl = t.co & kCoLds;
    it.o = (int)(t.co & (kTileAds - 1));
    it.w = (int)t.w;
    it.valid = 0u;
    uint32_t idx[kUserChunk];
    #pragma unroll
    for (int j = 0; j < kUserChunk; ++j) {
        it.valid |= (uint32_t)j < cnt ? (1u << j) : 0u;
        idx[j] = t.u0 + (uint32_t)j;
    }
    users_load<SRC>(a, lds_users, idx, it.valid, fl, it.ue);
    return it;
}

// One (query, posting) pair: round(fl(m' * w')) into the query's cell (users hold the row's
// cell code (acc_row_code) and m' bits, bucket entries w' bits). A cold pair of split buckets
// arrives as m' = 1 and w' = its rounded term, which this reproduces exactly.
template <bool W64>
__device__ __forceinline__ void pair_add(AccT<W64>* acc, uint2 ue, int o, int w) {
    const float p = __uint_as_float(ue.y) * __uint_as_float((uint32_t)w);
    const uint32_t byte = (ue.x & 0xffffu) + (((uint32_t)o << (W64 ? 5 : 4)) ^ (ue.x >> 16));
    AccT<W64>* cell = reinterpret_cast<AccT<W64>*>(reinterpret_cast<char*>(acc) + byte);
    if constexpr (W64)
        atomicAdd(cell, (unsigned long long)f32_to_i64_rn(p));
    else
        atomicAdd(cell, (uint32_t)__float2int_rn(p));
}

// The item's pairs, without a branch: a pair outside the item adds 0 to a cell of its own
// lane. With a branch per pair the compiler waited for all LDS operations in each branch, so
// every add waited for the one before it; a wave-uniform exit after the last used slot brings
// those waits back as well.
template <bool W64>
__device__ __forceinline__ void item_add(AccT<W64>* acc, const ItemLoad& it) {
    const uint32_t spare = (uint32_t)lane_id() * (uint32_t)sizeof(AccT<W64>);
    const uint32_t os = (uint32_t)it.o << (W64 ? 5 : 4);
    #pragma unroll
    for (int j = 0; j < kUserChunk; ++j) {
        const bool v = (it.valid >> j) & 1u;
        const uint2 ue = it.ue[j];
        const float p = __uint_as_float(ue.y) * __uint_as_float((uint32_t)it.w);
        const uint32_t byte = v ? (ue.x & 0xffffu) + (os ^ (ue.x >> 16)) : spare;
        AccT<W64>* cell = reinterpret_cast<AccT<W64>*>(reinterpret_cast<char*>(acc) + byte);
        if constexpr (W64)
            atomicAdd(cell, v ? (unsigned long long)f32_to_i64_rn(p) : 0ull);
        else
            atomicAdd(cell, v ? (uint32_t)__float2int_rn(p) : 0u);
    }
}

// Items of steps [s_begin, end) of a set of entries.
template <int SRC, bool W64>
__device__ __forceinline__ void item_steps(const ScoreArgs& a, const EntryItems& t, uint32_t s_begin,
                                           int* mark, AccT<W64>* acc, lds_uint2* lds_users) {
    if (s_begin == 0 && __ballot(t.nch > 1u) == 0ull) {
        item_add<W64>(acc, own_item_load<SRC>(a, t, lds_users));
        return;
    }
    int carry = carry_before(t, s_begin);
    for (uint32_t s = s_begin; 64u * s < t.total; ++s) {
        const int m = step_owner(t, s, mark, carry);
        item_add<W64>(acc, item_load<SRC>(a, t, s, m, lds_users));
    }
}

// The first step (64 items) of a tile's round-0 entries, mapped and their users loaded one
// tile before the adds (the loads' latency then hides behind a whole tile).
struct ItemsAhead {
    ItemLoad it;
    uint32_t total;
};

template <int SRC>
__device__ __forceinline__ ItemsAhead items_ahead(const ScoreArgs& a, int g, uint2 e, bool valid, bool hot,
                                                  int* mark, lds_uint2* lds_users, lds_u32* s_hot) {
    const EntryItems t = entry_items<SRC>(a, g, e, valid, hot, s_hot);
    ItemsAhead ia;
    ia.total = t.total;
    if (__ballot(t.nch > 1u) == 0ull) {
        ia.it = own_item_load<SRC>(a, t, lds_users);
        return ia;
    }
    int carry = -1;
    const int m = t.total > 0u ? step_owner(t, 0, mark, carry) : -1;
    ia.it = item_load<SRC>(a, t, 0, m, lds_users);
    return ia;
}

// The tile's shared bucket range: split buckets [hot | warm) sub-ranges 0 and 1 of the tile,
// else the tile's whole range (mid = beg: no hot entries).
__device__ __forceinline__ Bounds prod_bounds(const ScoreArgs& a, uint32_t tile) {
    Bounds b;
    const bool split = a.n_sub > 1;
    const uint32_t* p = a.tile_off + (size_t)tile * (uint32_t)a.n_sub;
    const uint32_t x0 = p[0], x1 = p[1], x2 = p[split ? 2 : 1];
    b.beg = x0;
    b.mid = split ? x1 : x0;
    b.end = split ? x2 : x1;
    return b;
}

__device__ __forceinline__ ProdTile prod_entries(const ScoreArgs& a, const Bounds& b, int pw) {
    ProdTile t;
    t.b = b;
    // every lane loads (lanes past the tile's entries read entry 0): a prefetch in a branch,
    // or selected right after its load, would make the compiler wait for it at once
    const uint32_t ei = b.beg + (uint32_t)pw + kCrossWaves * (uint32_t)lane_id();
    t.e0 = reinterpret_cast<const uint2*>(a.bucket)[ei < b.end ? ei : 0u];
    return t;
}

// Cross term of one tile (this wave's share): the prefetched first step of round 0, the rest
// of round 0, then later rounds of entries.
template <int SRC, bool W64>
__device__ __forceinline__ void prod_tile(const ScoreArgs& a, int g, int pw, const ProdTile& t,
                                          const ItemsAhead& ia, int* mark, AccT<W64>* acc,
                                          lds_uint2* lds_users, lds_u32* s_hot) {
    const int lane = lane_id();
    const uint2* bucket = reinterpret_cast<const uint2*>(a.bucket);
    constexpr uint32_t kRound = kCrossWaves * 64u;
    const uint32_t first = t.b.beg + (uint32_t)pw;
    if (first >= t.b.end) return;
    item_add<W64>(acc, ia.it);
    if (ia.total > 64u) {
        const uint32_t e0 = first + kCrossWaves * (uint32_t)lane;
        item_steps<SRC, W64>(a, entry_items<SRC>(a, g, t.e0, e0 < t.b.end, e0 < t.b.mid, s_hot), 1u, mark, acc,
                             lds_users);
    }
    for (uint32_t base = first + kRound; base < t.b.end; base += kRound) {
        const uint32_t ei = base + kCrossWaves * (uint32_t)lane;
        const bool ok = ei < t.b.end;
        const uint2 v = bucket[ok ? ei : 0u];
        const uint2 e = ok ? v : make_uint2(0u, 0u);
        item_steps<SRC, W64>(a, entry_items<SRC>(a, g, e, ok, ei < t.b.mid, s_hot), 0u, mark, acc, lds_users);
    }
}

template <int SRC>
__device__ __forceinline__ ItemsAhead prod_ahead(const ScoreArgs& a, int g, int pw, const ProdTile& t,
                                                 int* mark, lds_uint2* lds_users, lds_u32* s_hot) {
    const uint32_t e0 = t.b.beg + (uint32_t)pw + kCrossWaves * (uint32_t)lane_id();
    return items_ahead<SRC>(a, g, t.e0, e0 < t.b.end, e0 < t.b.mid, mark, lds_users, s_hot);
}


typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Eight e4m3fn codes (little-endian in v) -> eight BF16 values packed as one 16-byte operand,
// two codes per conversion instruction (scale 1: exact, every e4m3 value is a BF16 value).
__device__ __forceinline__ f32x4 fp8x8_to_bf16x8(uint2 v) {
    const bf16x2 p0 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(v.x, 1.0f, false);
    const bf16x2 p1 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(v.x, 1.0f, true);
    const bf16x2 p2 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(v.y, 1.0f, false);
    const bf16x2 p3 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(v.y, 1.0f, true);
    return f32x4{__builtin_bit_cast(float, p0), __builtin_bit_cast(float, p1), __builtin_bit_cast(float, p2),
                 __builtin_bit_cast(float, p3)};
}

// LDS quad of the FP32 copy's 16-byte unit j of a tile (row-major: ad j / (D / 4), chunk
// c = j mod (D / 4)): quad c >> 1, lane ((c & 1) << 5 | ad) XOR 2 (c >> 1).
template <int D>
__device__ __forceinline__ int f32_slot_d(int j) {
    const int o = j / (D / 4), c = j % (D / 4), i = c >> 1;
    return i * 64 + ((((c & 1) << 5) | o) ^ (2 * i));
}

// Embedding copies the scan can stream (DT): 0 = FP32 (row-major; staged into the 32x32x2
// operand order in LDS), 1 = BF16 and
// 2 = FP8 (both in the 32x32x16 BF16 operand layout; FP8 is expanded to BF16 in LDS and its
// per-ad scale applied to the finished dot product).
template <int D, int DT> struct EmbStage {
    static constexpr int UNITS = DT == 0 ? (D / 8) * 64 : (D / 16) * 64;  // 16-byte LDS units
};

// One work-group per (query group, contiguous range of tiles), persistent over its range;
// iteration `it` has the consumers score tile it from LDS buffers [it & 1] (and clear the
// accumulators they read) while the producers fill buffers [(it + 1) & 1] with tile it + 1
// and prefetch ahead. Every wave executes exactly 2 + n_it barriers.
//
// Work-group ids are laid out for the 8 XCDs of the chip (consecutive ids go to consecutive
// XCDs): all query groups of one tile range run on the same XCD, so the range's embedding
// blocks and bucket entries are fetched from HBM once and then served by that XCD's L2.
template <int D, int MODE, int DT, bool W64>
__global__ __launch_bounds__((ScoreShape<D, W64>::NT), 1) void k_score(ScoreArgs a) {
    constexpr int NQ = D / 8;
    using Acc = AccT<W64>;
    constexpr int GQ = ScoreShape<D, W64>::GQ;
    constexpr int CW = ScoreShape<D, W64>::CW;
    constexpr int NT = ScoreShape<D, W64>::NT;
    constexpr int kUsersLds = ScoreShape<D, W64>::USERS_LDS;
    constexpr int UNITS = EmbStage<D, DT>::UNITS;
    constexpr int SPER = (UNITS + kStageThreads - 1) / kStageThreads;  // units per stager lane
    __shared__ __attribute__((aligned(16))) Acc s_acc[2][GQ * kTileAds];
    __shared__ f32x4 s_emb[2][NQ * 64];
    __shared__ __attribute__((aligned(16))) float s_escale[2][kTileAds];
    __shared__ __attribute__((aligned(16))) float s_qscale[GQ];
    __shared__ __attribute__((aligned(16))) float s_thr[GQ];
    __shared__ uint32_t s_thr_hi[GQ];
    __shared__ uint32_t s_thr_lo[GQ];
    // Candidate ring (collect pass): consumer wave w pushes the cells of iteration it that
    // reach their row's FP32 threshold, as (row << 5 | ad offset, score bits, cross-term cell
    // bits), into its slice of half it & 1 and stores their count. In iteration it + 1 the same
    // wave makes the exact (key, id) comparison and issues the global appends' atomics first,
    // and writes the candidates at the end, so their latency hides behind the tile's work.
    __shared__ uint32_t s_ring[2][CW][kRingSlice][3];
    __shared__ uint32_t s_ring_n[2][CW];
    __shared__ int s_mark[kCrossWaves][64];
    __shared__ uint2 s_users[kUsersLds];
    __shared__ uint32_t s_hot[kHotMax];

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

    for (int i = tid; i < 2 * GQ * kTileAds; i += NT) (&s_acc[0][0])[i] = 0;
    if (tid < 2 * CW) (&s_ring_n[0][0])[tid] = 0u;
    // one query group: its (query, multiplier) users fit in LDS when few enough; split
    // buckets: this group's users of the hot keys (they fit by construction) and the hot-key
    // table
    const bool split = a.n_sub > 1;
    const bool users_in_lds = a.packed && a.n_users <= (uint32_t)kUsersLds;
    lds_uint2* lu = (lds_uint2*)s_users;
    lds_u32* lh = (lds_u32*)s_hot;
    if (users_in_lds) {
        for (uint32_t i = (uint32_t)tid; i < a.n_users; i += (uint32_t)NT)
            s_users[i] = reinterpret_cast<const uint2*>(a.users)[i];
    } else if (split) {
        const uint32_t h0 = a.hot_users_off[g], h1 = a.hot_users_off[g + 1];
        for (uint32_t i = (uint32_t)tid; i < h1 - h0; i += (uint32_t)NT)
            s_users[i] = reinterpret_cast<const uint2*>(a.hot_users)[h0 + i];
        for (int i = tid; i < a.n_hot; i += NT) s_hot[i] = a.hot_tab[(size_t)g * (uint32_t)a.n_hot + (uint32_t)i];
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
        }
    }
    auto tile_at = [&](int i) -> uint32_t {
        const int w = first + i;
        return MODE == 1 ? a.tile_list[w] : (uint32_t)w;  // the sample pass walks a tile list
    };
    __syncthreads();

    if (producer) {
        const int pw = wave - CW;
        if (pw < kStageWaves) {
            // Stager wave: the embedding block (and FP8 row scales) of tile u is loaded into
            // registers two iterations before the consumers read it and written to LDS one
            // iteration before; two register sets, for odd and even u. Its other loads are the
            // cold pairs of split buckets, issued in the same order as the blocks, so each wait
            // covers what the step needs and leaves the later tiles' loads in flight.
            const int sl = pw * 64 + lane;
            struct Raw {
                f32x4 u[SPER];   // FP32 / BF16 units
                uint2 c[SPER];   // FP8 codes
                float scale;     // FP8: the scale of ad sl of the tile
            };
            auto emb_load = [&](uint32_t t, Raw& r) {
                #pragma unroll
                for (int k = 0; k < SPER; ++k) {
                    const int j = sl + k * kStageThreads;
                    if (j < UNITS) {
                        if (DT == 2) r.c[k] = reinterpret_cast<const uint2*>(a.emb)[(int64_t)t * UNITS + j];
                        else r.u[k] = reinterpret_cast<const f32x4*>(a.emb)[(int64_t)t * UNITS + j];
                    }
                }
                if (DT == 2) r.scale = a.fp8_scale[(int64_t)t * kTileAds + (sl & (kTileAds - 1))];
            };
            auto emb_store = [&](int buf, const Raw& r) {
                #pragma unroll
                for (int k = 0; k < SPER; ++k) {
                    const int j = sl + k * kStageThreads;
                    if (UNITS % kStageThreads == 0 || j < UNITS) {
                        if (DT == 0) s_emb[buf][f32_slot_d<D>(j)] = r.u[k];
                        else s_emb[buf][j] = DT == 2 ? fp8x8_to_bf16x8(r.c[k]) : r.u[k];
                    }
                }
                if (DT == 2 && sl < kTileAds) s_escale[buf][sl] = r.scale;
            };
            // Split buckets: this group's cold pairs of tile u (their terms precomputed) are
            // added to the accumulators of tile u in the interval in which the cross-term waves
            // fill them; a tile's cold range is loaded two tiles ahead, its first 64 entries one
            // tile ahead (the rest, if any, when they are added).
            const uint2* bucket = reinterpret_cast<const uint2*>(a.bucket);
            struct Cold {
                uint2 b;  // the tile's cold range
                uint2 e;  // this lane's entry b.x + lane of it
            };
            auto cold_bounds = [&](int u) -> uint2 {
                const uint32_t* p = a.tile_off + (size_t)tile_at(u) * (uint32_t)a.n_sub + 2u + (uint32_t)g;
                return make_uint2(p[0], p[1]);
            };
            auto cold_entry = [&](uint2 b) -> uint2 {
                const uint32_t i = b.x + (uint32_t)lane;
                const uint2 v = bucket[i < b.y ? i : 0u];
                return i < b.y ? v : make_uint2(0u, 0u);
            };
            auto cold_pair = [&](Acc* acc, uint2 e) {  // (row << 5 | ad offset, term): m' = 1
                pair_add<W64>(acc, make_uint2(acc_row_code(e.x >> kTileShift, W64), 0x3f800000u),
                              (int)(e.x & (kTileAds - 1)), (int)e.y);
            };
            auto cold_add = [&](int buf, const Cold& c) {
                Acc* acc = s_acc[buf];
                if (c.b.x + (uint32_t)lane < c.b.y) cold_pair(acc, c.e);
                for (uint32_t i = c.b.x + 64u + (uint32_t)lane; i < c.b.y; i += 64u) cold_pair(acc, bucket[i]);
            };
            Cold cc{};
            uint2 cnb{};
            Raw ro, re;
            emb_load(tile_at(0), ro);
            if (split) {
                cc.b = cold_bounds(0);
                cc.e = cold_entry(cc.b);
                cold_add(0, cc);
                cc.b = cold_bounds(min(1, n_it - 1));
                cc.e = cold_entry(cc.b);
                cnb = cold_bounds(min(2, n_it - 1));
            }
            emb_store(0, ro);
            emb_load(tile_at(min(1, n_it - 1)), ro);
            emb_load(tile_at(min(2, n_it - 1)), re);
            __syncthreads();
            // The steady state has one path: past the range the loads repeat the last tile
            // (never used), and an odd last step is peeled off the loop, so that the compiler
            // counts the loads in flight exactly and waits only for the set being stored.
            auto step = [&](int u, Raw& r) {
                emb_store(u & 1, r);
                if (split) {
                    cold_add(u & 1, cc);
                    cc.b = cnb;
                    cc.e = cold_entry(cc.b);
                    cnb = cold_bounds(min(u + 2, n_it - 1));
                }
                emb_load(tile_at(min(u + 2, n_it - 1)), r);
                __syncthreads();
            };
            int u = 1;
            for (; u + 1 < n_it; u += 2) {
                step(u, ro);
                step(u + 1, re);
            }
            if (u < n_it) step(u, ro);
            __syncthreads();  // the consumers' last iteration
            return;
        }
        // Cross-term waves (instantiated per users source: LDS, global memory, or per entry
        // for split buckets): bucket bounds 64 tiles ahead, entries four tiles ahead, the
        // first step of items (mapped, users loaded) two tiles ahead.
        const int xw = pw - kStageWaves;
        auto cross = [&](auto src_tag) {
            constexpr int SRC = decltype(src_tag)::value;
            int* mark = s_mark[xw];
            // Bucket bounds of 64 consecutive tiles are held one tile per lane and read with
            // readlane; the next 64 tiles' are loaded when the current ones start being used,
            // so no per-tile chain of dependent loads waits on memory.
            struct BoundsBatch {
                uint32_t beg, mid, end;
            };
            auto bounds_batch = [&](int c) {  // lane i: tile slot 64 c + i (lanes past the range:
                                               // the last tile, never read)
                const Bounds b = prod_bounds(a, tile_at(min(64 * c + lane, n_it - 1)));
                return BoundsBatch{b.beg, b.mid, b.end};
            };
            BoundsBatch bcur = bounds_batch(0), bnxt = bounds_batch(1);
            int bc = 0;
            auto bounds_of = [&](int u) {  // u wave-uniform, never below the current batch
                if ((u >> 6) > bc) {
                    bcur = bnxt;
                    ++bc;
                    bnxt = bounds_batch(bc + 1);
                }
                const int i = u & 63;
                Bounds b;
                b.beg = (uint32_t)__builtin_amdgcn_readlane((int)bcur.beg, i);
                b.mid = (uint32_t)__builtin_amdgcn_readlane((int)bcur.mid, i);
                b.end = (uint32_t)__builtin_amdgcn_readlane((int)bcur.end, i);
                return b;
            };
            auto entries_of = [&](int u) { return prod_entries(a, bounds_of(u), xw); };
            {
                const ProdTile p0 = entries_of(0);
                prod_tile<SRC, W64>(a, g, xw, p0, prod_ahead<SRC>(a, g, xw, p0, mark, lu, lh), mark, s_acc[0], lu, lh);
            }
            // Tiles u = 1 .. n_it - 1 are filled in iteration u - 1, with the state kept in two
            // sets (odd and even u). Before the step for tile u its set holds: the first items
            // of u (mapped, loaded) and the entries of u, u + 2 and u + 4.
            struct Set {
                ItemsAhead pa;
                ProdTile pc, pn, pnn;
            };
            Set so{}, se{};
            // Past the range every stage works on the last tile again (never added), so the
            // steady state has one path and the compiler counts the loads in flight exactly.
            auto cl = [&](int u) { return min(u, n_it - 1); };
            auto fill = [&](Set& st, int u) {  // prologue: the state before the step for tile u
                st.pc = entries_of(cl(u));
                st.pa = prod_ahead<SRC>(a, g, xw, st.pc, mark, lu, lh);
                st.pn = entries_of(cl(u + 2));
                st.pnn = entries_of(cl(u + 4));
            };
            fill(so, 1);
            fill(se, 2);
            __syncthreads();
            auto step = [&](int u, Set& st) {
                const int nb = u & 1;  // buffer of tile u (the consumers read it in iteration u)
                prod_tile<SRC, W64>(a, g, xw, st.pc, st.pa, mark, s_acc[nb], lu, lh);
                st.pa = prod_ahead<SRC>(a, g, xw, st.pn, mark, lu, lh);
                st.pc = st.pn;
                st.pn = st.pnn;
                st.pnn = entries_of(cl(u + 6));
                __syncthreads();
            };
            int u = 1;
            for (; u + 1 < n_it; u += 2) {
                step(u, so);
                step(u + 1, se);
            }
            if (u < n_it) step(u, so);
            __syncthreads();  // the consumers' last iteration
        };
        if (split) cross(std::integral_constant<int, kSrcMixed>{});
        else if (users_in_lds) cross(std::integral_constant<int, kSrcLds>{});
        else cross(std::integral_constant<int, kSrcGlobal>{});
        return;
    }

    // consumer, groups of at most 2 CW queries (FP32, d <= 64): lane (wave w, half h) owns the
    // cell of row 2 w + h and ad column lane mod 32 and computes its dot product as a chain of
    // FMAs in the order and rounding of the 32x32x2 matrix product (per step the k = 0
    // dimension, then the k = 1 one, each rounded), so its scores are bit-identical to the
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
        auto iter = [&](int it) {
            if (wave_on) {
                const int cur = it & 1;
                Acc* acc = s_acc[cur];
                const f32x4* eb = s_emb[cur];
                float deep = 0.0f;
#pragma unroll
                for (int i = 0; i < NQ; ++i) {
                    const f32x4 e0 = eb[i * 64 + (o ^ (2 * i))];         // dimensions 8 i + j
                    const f32x4 e1 = eb[i * 64 + ((32 + o) ^ (2 * i))];  // dimensions 8 i + 4 + j
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        deep = fmaf(us[8 * i + j], e0[j], deep);
                        deep = fmaf(us[8 * i + 4 + j], e1[j], deep);
                    }
                }
                const int cell = acc_idx(row, o);
                const float wv = acc_value(acc[cell]);
                acc[cell] = 0;
                const float sq = s_qscale[row];
                const float sc = fmaf(wv, sq, deep);
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
                        if (key_passes(key, idk, s_thr_hi[row], s_thr_lo[row]))
                            append_candidate(a.cand, a.cand_cnt, a.cand_wide, a.cap, q, key, idk,
                                             wv * sq);
                    }
                }
            }
            __syncthreads();
        };
        for (int it = 0; it < n_it; ++it) iter(it);
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
            // step s = 4 i + j, k = lane >> 5: dimension 8 i + 4 k + j (the FP32 layout's order)
            const int kofs = lane >> 5;
            #pragma unroll
            for (int s = 0; s < NUR; ++s)
                ureg[s] = (q < B) ? a.user[(int64_t)q * D + 8 * (s >> 2) + 4 * kofs + (s & 3)] : 0.0f;
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
    bool wave_live = false;  // some query of this wave's 32 rows takes part in this pass
    {
        const int q = q0 + (lane & 31);
        wave_live = __ballot(q < B && (MODE != 0 || a.active[q] != 0u)) != 0ull;
    }
    __syncthreads();

    // Appends of this wave's ring slice of iteration it (entry `lane`): exact comparison with
    // the row's (key, id) threshold, then the atomic that reserves the slot; the candidate is
    // written by drain_finish, once the slot has returned.
    struct Pending {
        int q;
        uint32_t key, idk, pos;
        float wide;
        bool ok;
    };
    auto drain_issue = [&](int it) {
        Pending p{};
        const int h = it & 1;
        int l = lane;
        __asm__ volatile("" : "+v"(l));  // the slot address is computed here, not kept live
        const int wv = __builtin_amdgcn_readfirstlane(wave);  // wave-uniform: scalar address math
        if ((uint32_t)l < s_ring_n[h][wv]) {
            const uint32_t* e = s_ring[h][wv][l];
            const uint32_t x = e[0];
            const int ql = (int)(x >> kTileShift);
            const uint32_t key = score_key(__uint_as_float(e[1]));
            const uint32_t idk = 0xffffffffu - (uint32_t)((int64_t)tile_at(it) * kTileAds + (x & (kTileAds - 1)));
            if (key_passes(key, idk, s_thr_hi[ql], s_thr_lo[ql])) {
                p.q = qbase + ql;
                p.key = key;
                p.idk = idk;
                p.wide = __uint_as_float(e[2]) * s_qscale[ql];
                p.pos = atomicAdd(&a.cand_cnt[p.q], 1u);
                p.ok = true;
            }
        }
        return p;
    };
    auto drain_finish = [&](const Pending& p) {
        if (p.ok && p.pos < (uint32_t)a.cap) {
            a.cand[(int64_t)p.q * a.cap + p.pos] = ((unsigned long long)p.key << 32) | (unsigned long long)p.idk;
            if (a.cand_wide) a.cand_wide[(int64_t)p.q * a.cap + p.pos] = p.wide;
        }
    };
    // this lane's rows: group g4 (0..3) holds rows rg(g4) .. rg(g4) + 3 of the group's 256
    auto rg = [&](int g4) { return wave * 32 + 8 * g4 + 4 * (lane >> 5); };
    const int o = lane & 31;
    auto iter = [&](int it) {
        const int cur = it & 1;
        Acc* acc = s_acc[cur];
        if (!wave_live) {
            // rows of queries in the batch but inactive in this round still receive cross
            // terms: keep the buffer clear for its next use. Rows past the batch are never
            // written (the buffers start cleared), so their waves only keep the barrier count.
            if (q0 < B) {
                #pragma unroll
                for (int g4 = 0; g4 < 4; ++g4) clear4(acc + acc_idx(rg(g4), o));
            }
            __syncthreads();
            return;
        }
        // the survivors of iteration it - 1: their appends' atomics are issued now
        Pending pd{};
        if (MODE == 0 && it > 0) pd = drain_issue(it - 1);
        // products first: the tile's B operands are read from LDS up to eight quads ahead of
        // the products that use them, so one LDS latency is exposed per tile
        const uint32_t tile = tile_at(it);
        f32x16 c = {};
        const f32x4* eb = s_emb[cur];
        if (DT == 0) {
            constexpr int W = NQ < 8 ? NQ : 8;
            f32x4 ev[W];
            #pragma unroll
            for (int i = 0; i < W; ++i) ev[i] = eb[i * 64 + (lane ^ (2 * i))];
            #pragma unroll
            for (int i = 0; i < NQ; ++i) {
                const f32x4 e4 = ev[i % W];
                if (i + W < NQ) ev[i % W] = eb[(i + W) * 64 + (lane ^ (2 * (i + W)))];
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
        float wd[16];  // the row's scale is applied below
        {
            Acc av[16];
            #pragma unroll
            for (int g4 = 0; g4 < 4; ++g4) read4(acc + acc_idx(rg(g4), o), av + 4 * g4);
            #pragma unroll
            for (int g4 = 0; g4 < 4; ++g4) clear4(acc + acc_idx(rg(g4), o));
            #pragma unroll
            for (int r = 0; r < 16; ++r) wd[r] = acc_value(av[r]);
        }
        const float escale = DT == 2 ? s_escale[cur][o] : 1.0f;
        const int64_t ad = (int64_t)tile * kTileAds + o;
        const bool ad_ok = ad < a.n_ads;
        float sc[16];
        // some cell of the wave is at or above its row's FP32 threshold: each comparison's
        // lane mask (one vector compare into scalar registers), or-ed on the scalar unit
        const uint64_t okm = __ballot(ad_ok);
        uint64_t any = 0;
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
                    any |= __ballot(sc[4 * g4 + k] >= th[k]);  // NaN threshold: never
                }
            }
        }
        if (MODE == 0) {
            // rare: push this wave's cells at or above the FP32 threshold into its ring slice
            // (the stager makes the exact comparison); a full slice appends directly
            uint32_t n = 0;  // wave-uniform
            if ((any & okm) != 0ull) {
                f32x4 thv[4];  // the rows' thresholds again, read together
                #pragma unroll
                for (int g4 = 0; g4 < 4; ++g4) thv[g4] = *reinterpret_cast<const f32x4*>(s_thr + rg(g4));
                #pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const bool mine = ad_ok && sc[r] >= thv[r >> 2][r & 3];
                    const uint64_t bl = __ballot(mine);
                    if (bl == 0ull) continue;
                    if (mine) {
                        int ql = wave * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                        __asm__ volatile("" : "+v"(ql));  // per-row addresses computed here, not hoisted
                        const uint32_t slot = n + (uint32_t)__builtin_amdgcn_mbcnt_hi(
                                                          (uint32_t)(bl >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bl, 0u));
                        if (slot < (uint32_t)kRingSlice) {
                            uint32_t* e = s_ring[cur][wave][slot];
                            e[0] = ((uint32_t)ql << kTileShift) | (uint32_t)o;
                            e[1] = __float_as_uint(sc[r]);
                            e[2] = __float_as_uint(wd[r]);
                        } else {
                            const uint32_t key = score_key(sc[r]);
                            const uint32_t idk = 0xffffffffu - (uint32_t)ad;
                            if (key_passes(key, idk, s_thr_hi[ql], s_thr_lo[ql]))
                                append_candidate(a.cand, a.cand_cnt, a.cand_wide, a.cap, qbase + ql, key, idk,
                                                 wd[r] * s_qscale[ql]);
                        }
                    }
                    n += (uint32_t)__builtin_popcountll(bl);
                }
            }
            if (lane == 0) s_ring_n[cur][wave] = min(n, (uint32_t)kRingSlice);
            drain_finish(pd);
        }
        __syncthreads();
    };
    for (int it = 0; it < n_it; ++it) iter(it);
    if (MODE == 0 && wave_live) drain_finish(drain_issue(n_it - 1));
}

// Exact FP32 rescore of the Kc approximate-best candidates of query q (one work-group): each
// candidate's FP32 row (row-major copy) is gathered by one thread, whose dot product is the
// FP32 scan's own FMA chain, so the rescored score is bit-identical to the FP32 scan's; the
// score adds the carried cross term. The K best exact keys are found by radix select, sorted
// and written. Certificate:
// every ad outside the candidates has an approximate score <= the Kc-th approximate score s~
// and differs from its exact score by at most eps_q, so s~ + eps_q < (K-th exact score)
// proves the result is the exact top-K; otherwise the query is marked uncertified.
template <int D>
__global__ __launch_bounds__(1024) void k_rescore(RescoreArgs a) {
    constexpr int NQ = D / 8;
    __shared__ unsigned long long s[kMaxK];
    __shared__ float s_u[D];
    __shared__ uint32_t s_hist[256];
    __shared__ unsigned long long s_pref;
    __shared__ int s_rank;
    __shared__ uint32_t s_slot;
    const int q = (int)blockIdx.x;
    const int tid = (int)threadIdx.x;
    const int K = a.kq[q];
    if (a.ctl && a.ctl->error) return;
    if (a.skip && *a.skip != 0u) return;
    if (K <= 0 || a.status[q] != kStatusDone) return;
    const int Kc = a.kcnt[q];
    for (int i = tid; i < D; i += 1024) s_u[i] = a.user[(int64_t)q * D + i];
    __syncthreads();
    // one thread per candidate: the dot product is one FMA chain over the dimensions in the
    // order the FP32 scan's 32x32x2 products take them (per step s = 4 i + j dimension 8 i + j,
    // then 8 i + 4 + j, each rounded), so a rescored score has the FP32 scan's bits; the cross
    // term is the scan's exact value.
    const f32x4* emb = reinterpret_cast<const f32x4*>(a.emb);
    for (int r = tid; r < Kc; r += 1024) {
        uint32_t id = a.r_id[(int64_t)q * a.r_ld + r];
        if ((int64_t)id >= a.n_ads) {  // never from a correct scan: report, read a valid row
            if (a.ctl) atomicOr(&a.ctl->error, 4u);
            id = 0u;
        }
        const f32x4* row = emb + (int64_t)id * (D / 4);  // the ad's row: 2 x 128-byte lines (d = 64)
        f32x4 e0[NQ], e1[NQ];
        #pragma unroll
        for (int i = 0; i < NQ; ++i) {
            e0[i] = row[2 * i];      // dimensions 8 i + j
            e1[i] = row[2 * i + 1];  // dimensions 8 i + 4 + j
        }
        float deep = 0.0f;
        #pragma unroll
        for (int i = 0; i < NQ; ++i) {
            #pragma unroll
            for (int j = 0; j < 4; ++j) {
                deep = fmaf(s_u[8 * i + j], e0[i][j], deep);
                deep = fmaf(s_u[8 * i + 4 + j], e1[i][j], deep);
            }
        }
        const float sc = deep + a.r_wide[(int64_t)q * a.r_ld + r];
        s[r] = ((unsigned long long)score_key(sc) << 32) | (unsigned long long)(0xffffffffu - id);
    }
    // the K best exact keys, sorted: the K-th best by radix select, the keys at or above it
    // (exactly K: they are distinct) moved to the front, then a sort of those alone
    if (tid == 0) s_slot = 0u;
    __syncthreads();
    const unsigned long long T = kth_largest(s, Kc, K, s_hist, &s_pref, &s_rank);
    {
        constexpr int R = kMaxK / 1024;
        unsigned long long v[R];
        #pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = tid + 1024 * i;
            v[i] = r < Kc ? s[r] : 0ull;
        }
        __syncthreads();
        #pragma unroll
        for (int i = 0; i < R; ++i)
            if (tid + 1024 * i < Kc && v[i] >= T) s[atomicAdd(&s_slot, 1u)] = v[i];
    }
    int P = 64;
    while (P < K) P <<= 1;
    for (int i = K + tid; i < P; i += 1024) s[i] = 0ull;
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
        } else if (a.werr && !wide_precise(a.werr[q], key_score((uint32_t)(s[0] >> 32)),
                                           key_score((uint32_t)(s[K - 1] >> 32)))) {
            a.status[q] = kStatusImprecise;
            atomicAdd(a.imprecise, 1u);
        }
    }
}

template <int D, int DT, bool W64>
static void launch_score_dt(const ScoreArgs& a, int mode, dim3 grid, hipStream_t st) {
    constexpr int NT = ScoreShape<D, W64>::NT;
    if (mode == 0) hipLaunchKernelGGL((k_score<D, 0, DT, W64>), grid, dim3(NT), 0, st, a);
    else if (mode == 1) hipLaunchKernelGGL((k_score<D, 1, DT, W64>), grid, dim3(NT), 0, st, a);
    else hipLaunchKernelGGL((k_score<D, 2, DT, W64>), grid, dim3(NT), 0, st, a);
}

// 64-bit cells only for FP32 scans (the rerun of queries whose 32-bit quantum is too coarse,
// and callers that ask for them).
template <int D>
void launch_score_d(const ScoreArgs& a, int mode, int dt, dim3 grid, hipStream_t st) {
    if (dt == 0) {
        if (a.wide64) launch_score_dt<D, 0, true>(a, mode, grid, st);
        else launch_score_dt<D, 0, false>(a, mode, grid, st);
    } else if (dt == 1) {
        launch_score_dt<D, 1, false>(a, mode, grid, st);
    } else {
        launch_score_dt<D, 2, false>(a, mode, grid, st);
    }
}

template <int D>
void launch_rescore_d(const RescoreArgs& a, int n_queries, hipStream_t st) {
    hipLaunchKernelGGL(k_rescore<D>, dim3((unsigned)n_queries), dim3(1024), 0, st, a);
}

}  // namespace ebr
