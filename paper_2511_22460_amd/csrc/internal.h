// Internal declarations shared by the host runtime and the gfx950 kernels of libebr.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ebr.h"

namespace ebr {

// ---------------------------------------------------------------- layout constants

// Ads per tile: one 32-wide column block of the 32x32 matrix-core tile, and the
// unit of the tile-major posting buckets built per batch.
constexpr int kTileAds = 32;
constexpr int kTileShift = 5;
// Ads per super-tile: the unit of the first bucketing pass of a batch's postings.
constexpr int kSuperAds = 1024;
constexpr int kSuperShift = 10;
constexpr int kTilesPerSuper = kSuperAds / kTileAds;
// Super-tiles of a batch without split buckets: 2048 ads (fewer, longer runs per list).
constexpr int kMaxSuperShift = 11;
// Postings per compressed chunk: one per lane of a 64-wide wavefront.
constexpr int kChunk = 64;
// Candidate slots per query in the selection buffer (sorted in LDS at the end).
constexpr int kCandCap = 16384;
// Largest K a query may ask for.
constexpr int kMaxK = 8192;

// One compressed chunk of up to 64 postings of one key.
//  first_id  id of posting 0
//  info      bits 0..5: gap width b (0..32); bits 8..14: count (1..64)
//  word_off  first 32-bit word of the packed gaps in the index's word array
//  post_off  index of posting 0 in the weight array
// Gaps g_i = id_i - id_{i-1} - 1 (i = 1..count-1) are stored LSB-first, b bits
// each, starting at bit 0 of word word_off.
struct ChunkHdr {
    uint32_t first_id;
    uint32_t info;
    uint32_t word_off;
    uint32_t post_off;
};
static_assert(sizeof(ChunkHdr) == 16, "chunk header is 16 bytes");

inline int hdr_bits(uint32_t info) { return (int)(info & 63u); }
inline int hdr_count(uint32_t info) { return (int)((info >> 8) & 127u); }

// ---------------------------------------------------------------- host-side index

struct Index {
    int64_t n_ads = 0, n_keys = 0, n_postings = 0, n_chunks = 0;
    int32_t dim = 0;
    int64_t n_tiles = 0;      // ceil(n_ads / 32)
    uint32_t dtypes = 0;
    // device pointers into the caller's arena
    const void* emb_f32 = nullptr;   // row-major, padded to whole tiles (see k_score in score.h)
    const void* emb_bf16 = nullptr;  // 32x32x16 BF16 operand layout (optional)
    const void* emb_fp8 = nullptr;   // same element order, e4m3fn codes (optional)
    const float* fp8_scale = nullptr;  // per ad row (optional)
    // quantisation error summaries for the recall certificate, per copy (0 = BF16, 1 = FP8):
    // max_a ||e_a - e^_a||_2 and max_a ||e^_a||_2; and max_a ||e_a||_2 of the FP32 rows
    double q_err2[2] = {0.0, 0.0}, q_norm2[2] = {0.0, 0.0}, e_norm2 = 0.0;
    const ChunkHdr* chunks = nullptr;
    const uint32_t* words = nullptr;
    const float* weights = nullptr;  // null: an ids-only index (every weight 1)
    // host copies for planning
    std::vector<uint32_t> key_chunk_off;  // V + 1
    std::vector<int64_t> key_post_off;    // V + 1
    std::vector<float> key_maxw;          // V, max |w| of each list
    std::vector<int8_t> key_wshift;       // V, Sw_k: weights of key k enter sums as w * 2^Sw_k
    ebr_index_info stats{};
    int device = 0;
    // launch shapes recorded by the autotuner, per (scan dtype, query groups)
    mutable std::mutex shape_mu;
    std::map<std::pair<int, int>, ebr_launch_shape> shapes;
};

// Arena plan: byte offsets of each section (256-byte aligned).
struct ArenaPlan {
    size_t off_emb_f32 = 0, off_chunks = 0, off_words = 0, off_weights = 0, total = 0;
    size_t bytes_emb_f32 = 0, bytes_chunks = 0, bytes_words = 0, bytes_weights = 0;
    size_t off_emb_bf16 = 0, off_emb_fp8 = 0, off_fp8_scale = 0;
    size_t bytes_emb_bf16 = 0, bytes_emb_fp8 = 0, bytes_fp8_scale = 0;
    int64_t n_chunks = 0, n_words = 0;
};

// Arena sections of an index of these sizes (n_chunks 64-posting chunks, n_words packed gap
// words; weights: whether a weight array is stored).
ArenaPlan arena_plan(int64_t n_ads, int32_t dim, uint32_t dtypes, int64_t n_post, int64_t n_chunks,
                     int64_t n_words, bool weights);

// ---------------------------------------------------------------- error plumbing

void set_error(const char* fmt, ...);
const char* last_error();

// ---------------------------------------------------------------- codec (host)

// Number of chunks and packed words a list of n ids occupies.
void codec_measure(const uint32_t* ids, int64_t n, int64_t* chunks, int64_t* words);
// Encode one list: hdr receives ceil(n/64) headers (word_off relative to
// word_base, post_off relative to post_base), words receives the packed gaps.
void codec_encode(const uint32_t* ids, int64_t n, ChunkHdr* hdr, uint32_t* words,
                  uint32_t word_base, uint32_t post_base);
// Decode one list encoded with word_base = post_base = 0.
bool codec_decode(const ChunkHdr* hdr, int64_t n_chunks, const uint32_t* words,
                  int64_t n_words, int64_t n, uint32_t* ids);

// ---------------------------------------------------------------- quantisers (quant.cpp)

uint16_t bf16_rne(float x);
float bf16_to_f32(uint16_t h);
uint8_t fp8_e4m3_rne(float x);
float fp8_e4m3_to_f32(uint8_t c);
// position of element (row a, dim k) in the 32x32x16 BF16 operand layout (elements)
size_t mfma16_index(int64_t a, int k, int d);

// ---------------------------------------------------------------- kernels

// Every launcher returns hipSuccess or the first HIP error (as int).
struct ScoreArgs;

int launch_swizzle_f32(const float* src_rows, int64_t n_rows, int64_t row0, int32_t dim,
                       void* dst, void* stream);

// ---------------------------------------------------------------- batches (api.cpp)

// The sizes a top-K batch's workspace depends on.
struct BatchSizes {
    int B = 0;
    int64_t nnz = 0;        // (query, feature) pairs
    int nu = 0;             // distinct keys
    uint64_t bucket_n = 0;  // postings of the distinct keys
    int kcmax = 0;          // largest K' (K, or the rescore factor times K) of the batch
    int64_t n_out = 0;      // sum of K
    int64_t n_sample = 0;   // sample tiles (derived; ignored by topk_workspace_bytes)
    int64_t big_n = 0;      // ads to sort for queries whose K exceeds the LDS sort (0: none)
};

// Exact workspace bytes of a top-K batch of these sizes on scan dtype `dtype`.
size_t topk_workspace_bytes(const Index& ix, int dtype, BatchSizes z);

// ebr_score_topk without the entry point's bookkeeping; stream is a hipStream_t. With a
// graph handle the device sequence is captured and launched as one graph
// (ebr_score_topk_graph); shape, when non-null, replaces the recorded launch shape.
ebr_status run_topk(const Index& ix, const ebr_batch* batch, char* ws, size_t ws_bytes,
                    uint32_t* out_ids, float* out_scores, void* stream, ebr_timings* tm,
                    ebr_graph* graph = nullptr, const ebr_launch_shape* shape = nullptr);

}  // namespace ebr

// The C-ABI handle is the index itself.
struct ebr_index : ebr::Index {};
