// Kernel argument blocks and launchers of libebr (host <-> device interface).
#pragma once

#include <cstdint>

#include "internal.h"

namespace ebr {

constexpr int kStatusDone = 0;
constexpr int kStatusPending = 1;
constexpr int kStatusNeedLower = 2;
constexpr int kStatusOverflow = 3;
constexpr int kStatusUncertified = 4;
constexpr int kStatusImprecise = 5;

// A 32-bit fixed-point cross term is accepted for a query when its worst-case rounding (half a
// quantum per feature) is at most this fraction of every returned score's magnitude: 2^-18,
// the worst-case relative error of a 64-term FP32 dot product (64 * 2^-24), a quarter of the
// 1e-5 tolerance. Queries that miss it are rerun with 64-bit cells.
constexpr float kWideTau = 0x1p-18f;

// Threshold-revision rounds enqueued per batch without host synchronisation; a round whose
// predecessor left no query unresolved exits at once.
constexpr int kMaxRounds = 4;

// Query groups of the scoring kernel (shared by the host planner and the kernel): queries per
// group, and the (query, multiplier) records one work-group keeps in LDS.
constexpr int score_gq(int dim, bool w64) { return (dim <= 64 && !w64) ? 256 : 128; }
constexpr int score_users_lds(int dim, bool w64) { return (dim > 64 && w64) ? 4096 : 8192; }

// Split buckets of a batch of several query groups. Its distinct keys are numbered hot, then
// warm, then cold:
//   hot  - the keys with the longest lists, as many as fit every group's LDS (at most kHotMax
//          keys; each group's users of them at most score_users_lds). Their postings are
//          shared by all groups; a work-group finds a key's users in an LDS table.
//   warm - other keys with more users than query groups: shared postings, users found through
//          the global users_off table.
//   cold - keys with at most as many users as query groups: one bucket entry per (posting,
//          user), carrying the pair's rounded term round(fl(m' w')) (an FP32 integer value),
//          in the bucket of the user's query group.
// Per tile the bucket holds [hot | warm | cold of group 0 | ... | cold of group G - 1], so the
// tile offsets have n_tiles * (G + 2) + 1 entries.
constexpr int kHotMax = 2048;
constexpr int kSplitMaxGroups = 62;
inline bool split_groups(int n_qg) { return n_qg > 1 && n_qg <= kSplitMaxGroups; }
inline int cold_user_limit(int n_qg) { return n_qg; }

// The cross-term cell of query row q (within its group) and ad offset o sits at byte
// B(q) + ((o << s) ^ X(q)) of the LDS accumulator tile, s = 4 for 32-bit and 5 for 64-bit cells
// (rows grouped by four, the column XOR-swizzled by the row group; the layout is acc_idx in
// score.h): B(q) = (q >> 2) 128 c + (q & 3) c and X(q) = ((q >> 2) & 31) << s with c the cell
// bytes. A user record carries code = B | X << 16 instead of its row, so that a pair's cell
// address is three instructions.
inline constexpr uint32_t acc_row_code(uint32_t q, bool w64) {
    return w64 ? (((q >> 2) * 1024u + (q & 3u) * 8u) | ((((q >> 2) & 31u) << 5) << 16))
               : (((q >> 2) * 512u + (q & 3u) * 4u) | ((((q >> 2) & 31u) << 4) << 16));
}

// Per-batch control block (device, in the workspace).
struct Control {
    uint32_t error;                   // bit 0: non-finite user row; bit 1: not converged;
                                      // bit 2: a rescore candidate id out of range
    uint32_t unres[kMaxRounds];       // queries left unresolved by round r
    uint32_t uncertified;             // reduced-precision scans: failed certificates
    uint32_t imprecise;               // queries whose 32-bit cross term missed kWideTau
    uint32_t pad[9];
};

struct DecodeArgs {
    const ChunkHdr* chunks;
    const uint32_t* words;
    const float* weights;             // null: an ids-only index (every weight 1)
    const uint32_t* uk_chunk_begin;   // per distinct key: its first chunk in the index
    const uint32_t* uk_chunk_prefix;  // n_ukeys + 1 prefix sums of chunk counts
    const int32_t* uk_wshift;         // per distinct key: Sw_k, weights enter sums as w * 2^Sw_k
    int32_t n_ukeys;
    uint32_t total_chunks;
    uint32_t chunks_per_wave;         // consecutive chunks one decode wavefront takes (1..64)
    int64_t n_tiles;
    int64_t n_super;                  // super-tiles of 2^sshift ads
    int32_t sshift;                   // 10 (1024 ads; always with split buckets) or
                                      // kMaxSuperShift (2048 ads)
    uint32_t* st_cnt;                 // count pass: postings per super-tile
    const uint32_t* st_off;           // n_super + 1 exclusive prefix
    uint32_t* st_fill;                // place pass: running fill per super-tile
    uint32_t* stage;                  // place pass: pairs ((slot << 10) | ad & 1023, w' bits)
    uint2* chunk_map;                 // per batch chunk: (slot, chunk index in the index)
    const uint32_t* users_off;        // non-null: final entries carry their key's users range
    uint32_t* tile_off;               // refine: n_tiles * n_sub + 1 offsets into bucket
    uint32_t* bucket;                 // refine: pairs (users range or slot | ad & 31, w' bits)
    // split buckets (n_sub = groups + 2; 1 otherwise)
    int32_t n_sub;
    int32_t n_hot;                    // slots [0, n_hot) are hot
    int32_t cold_first;               // slots [cold_first, n_ukeys) are cold
    int32_t gq_shift;                 // log2 of the queries per group
    const uint32_t* cold_off;         // per cold slot: its users in cold_users (CSR)
    const uint32_t* cold_users;       // pairs (query index in the batch, bits of m')
};

struct ScoreArgs {
    const void* emb;                  // the scanned embedding copy (layout per dtype)
    const float* fp8_scale;           // FP8 copy: per-ad scales
    int32_t dtype;                    // 0 FP32, 1 BF16, 2 FP8
    int64_t n_ads;
    const float* user;                // B x D
    int32_t n_queries;
    int32_t n_qgroups;
    int32_t packed;                   // bucket entries carry users ranges (one query group)
    int32_t wide64;                   // 64-bit cross-term cells (FP32 scans; 128-query groups)
    const uint32_t* tile_off;         // n_tiles * n_sub + 1
    const uint32_t* bucket;           // pairs
    int32_t n_sub;                    // sub-ranges per tile (split buckets: groups + 2)
    int32_t n_hot;                    // split buckets: hot keys
    const uint32_t* hot_tab;          // split: per (group, hot slot) (users index << 9) | count
    const uint32_t* hot_users;        // split: per group, its users of the hot keys
    const uint32_t* hot_users_off;    // split: groups + 1 offsets into hot_users
    const uint32_t* users_off;        // n_ukeys * n_qgroups + 1
    const uint32_t* users;            // pairs (query within group, bits of m')
    uint32_t n_users;                 // pairs in users
    const double* qinv;               // 2^-S per query
    int32_t n_work;                   // tiles to visit
    int32_t n_ranges;                 // contiguous tile ranges per query group (set at launch)
    const uint32_t* tile_list;        // null: tile = work index
    // collect mode
    const uint32_t* thresh;           // pairs (key hi, ~id lo) per query
    const uint32_t* active;           // per query
    unsigned long long* cand;         // B x cap
    float* cand_wide;                 // B x cap cross-term values (approximate scans), or null
    uint32_t* cand_cnt;               // B
    int32_t cap;
    // sample mode
    uint32_t* sample_keys;
    int64_t sample_ld;
    // dense mode
    float* deep_out;
    float* wide_out;
    // collect mode: run only if gate is null or *gate != 0, and never after an input error
    const uint32_t* gate;
    const Control* ctl;
};

struct SelectArgs {
    const uint32_t* keys;
    int64_t ld;
    int64_t n_cols;
    const int32_t* jq;
    const int32_t* kq;
    const int32_t* status;
    int32_t only_status;              // -1: every query with K > 0
    uint32_t* thresh;
    // revision rounds: run only if gate is null or *gate != 0; round 1 takes the kcnt-th
    // sample key (if the sample holds that many), later rounds no threshold at all
    const uint32_t* gate;
    int32_t round;
    const int32_t* kcnt;
    int64_t n_valid;
    const Control* ctl;
};

struct FinalArgs {
    uint32_t* active;
    const int32_t* kq;                // K per query
    const int32_t* kcnt;              // candidates to keep: K (output mode) or K' (prep mode)
    const uint32_t* cand_cnt;
    int32_t cap;
    const unsigned long long* cand;
    const float* cand_wide;           // prep mode
    int32_t* status;
    uint32_t* thresh;
    uint32_t* unresolved;
    int32_t prep;                     // 0: write the top K; 1: stage the top K' for the rescore
    const int64_t* out_off;
    uint32_t* out_ids;
    float* out_scores;
    const uint32_t* gate;             // run only if null or *gate != 0
    const Control* ctl;               // nothing is written after an input error
    const float* werr;                // output mode: per-query bound on the cross term's
                                      // fixed-point rounding, or null (no check)
    uint32_t* imprecise;              // count of queries that missed kWideTau
    uint32_t* r_id;                   // prep: B x r_ld ids of the Kc best, in no particular order
    float* r_wide;                    // prep: their cross-term values
    float* r_stilde;                  // prep: the K'-th approximate score per query
    int32_t r_ld;
};

struct RescoreArgs {
    const void* emb;                  // FP32 copy (row-major)
    const float* user;                // B x D
    int64_t n_ads;
    const int32_t* kq;
    const int32_t* kcnt;
    int32_t* status;
    uint32_t* uncertified;
    const uint32_t* r_id;
    const float* r_wide;
    const float* r_stilde;
    const float* eps;                 // per query: bound on |approximate - exact| score
    const float* werr;                // per query: cross-term rounding bound, or null
    uint32_t* imprecise;
    Control* ctl;                     // bit 2 of error: a candidate id outside the inventory
    const uint32_t* skip;             // non-null and nonzero: selection unfinished, do nothing
    int32_t r_ld;
    const int64_t* out_off;
    uint32_t* out_ids;
    float* out_scores;
};

// Per-query set-up on the device: user rows must be finite (else ctl->error bit 0), status
// and activity from K, and for reduced-precision scans the certificate's eps (see k_rescore).
struct PrepArgs {
    const float* user;
    int32_t n_queries;
    int32_t dim;
    const int32_t* kq;
    const double* aq;                 // per query: sum_j |m_j| max|W[k_j,:]|
    int32_t* status;
    uint32_t* active;
    float* eps;                       // null for FP32 scans
    double q_err2, q_norm2, e_norm2;  // the index's error summaries for the scanned copy
    Control* ctl;
};

int launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, void* stream);
int launch_prep(const PrepArgs& a, void* stream);
// Zero the candidate counts of round `round` (skipped when the gate is zero).
int launch_round_reset(uint32_t* cand_cnt, int32_t n, const uint32_t* gate, void* stream);
int64_t scan_tmp_words(int64_t n);
int launch_excl_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, void* stream);
// Per batch chunk, its distinct-key slot and index chunk (before the decode passes).
int launch_chunk_map(const DecodeArgs& a, void* stream);
int launch_decode(const DecodeArgs& a, int place, void* stream);
int launch_refine(const DecodeArgs& a, void* stream);
// Decode the chunks [chunk0, chunk0 + n_chunks) of consecutive keys: posting p (index into the
// index's posting order) goes to ids / w at p - post_base; null weights decode as 1.
int launch_decode_key(const ChunkHdr* chunks, const uint32_t* words, const float* weights,
                      uint32_t chunk0, uint32_t n_chunks, uint32_t post_base, uint32_t* ids,
                      float* w, void* stream);
bool score_dim_supported(int dim);
// Queries per query group of the scoring kernel for this embedding width and cell width.
inline int score_group_queries(int dim, bool wide64 = false) { return score_gq(dim, wide64); }
int score_ranges(int n_work, int n_qgroups, int ctas);
int launch_score(const ScoreArgs& a, int dim, int mode, int ranges, void* stream);
int launch_select(const SelectArgs& a, int n_queries, void* stream);
// Blocks of the full sort over n keys (its histogram holds 256 x blocks + 1 words).
int64_t sort_blocks(int64_t n);
// One query's top-K by a full sort of its n scores deep[a] + wide[a] (order: score descending,
// id ascending): keys and tmp hold n 64-bit keys each, hist 256 x sort_blocks(n) + 1 words,
// scan_tmp scan_tmp_words(256 x sort_blocks(n)) words; ids / scores receive K entries.
int launch_full_sort_topk(const float* deep, const float* wide, int64_t n, int64_t k,
                          unsigned long long* keys, unsigned long long* tmp, uint32_t* hist,
                          uint32_t* scan_tmp, uint32_t* ids, float* scores, void* stream);
int launch_finalize(const FinalArgs& a, int n_queries, void* stream);
int launch_rescore(const RescoreArgs& a, int dim, int n_queries, void* stream);

}  // namespace ebr
