/*
 * ebr.h - C ABI of libebr, an MI355X (gfx950) implementation of the retrieval
 * hot path of "An Efficient Embedding Based Ad Retrieval with GPU-Powered
 * Feature Interaction" (arXiv 2511.22460).
 *
 * For every query and every ad of the inventory the library computes
 *
 *     s(u, a) = <u, e_a> + sum_j m_j * W[k_j, a]
 *
 * and returns the K ads with the largest s, ordered by (s descending, ad id
 * ascending). The first term is the dual-tower inner product (Section 3.1,
 * equation "dual-tower"; IPNN-extended towers are the same product over longer
 * vectors, Section 3.2). The second is the HitMatch explicit cross term
 * (Section 3.3, equation "hitmatch"), served from an inverted list that maps
 * each user feature value (key) to the ids of the ads carrying it, the input
 * of the indexing algorithm of Section 3.4 (Algorithm 1). The
 * paper's binary L with per-feature weight w_i x_i is the case W == 1 (pass
 * post_w = NULL) with m_j = w_j x_j (feat_mult). The paper's query carries its
 * non-zero feature values {(k, w_hat)} (Algorithm 2, its input).
 *
 * Conventions for every call:
 *  - Return codes are ebr_status; EBR_OK is 0, errors are negative, and
 *    ebr_last_error() gives a thread-local message for the last failure.
 *  - No exception crosses the ABI. On error no output buffer is written.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *    memory of the device current at the call (for instance a torch tensor's
 *    data_ptr()). hip_stream is a hipStream_t (NULL = the null stream).
 *  - The library never allocates device memory: the index lives in a
 *    caller-owned arena, batch scratch in a caller-owned workspace, each sized
 *    by a *_size query. Both must outlive the objects that use them.
 *  - HIP failures map to EBR_EDEVICE with hipGetErrorString text.
 */
#ifndef EBR_H
#define EBR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EBR_OK = 0,
    EBR_EINVAL = -1,       /* invalid argument or input data */
    EBR_ENOMEM = -2,       /* arena / workspace / scratch budget too small */
    EBR_EDEVICE = -3,      /* HIP runtime or kernel failure */
    EBR_EAGAIN = -4,       /* not ready yet / queue full */
    EBR_ENOTFOUND = -5,    /* unknown ticket */
    EBR_ESHUTDOWN = -6,    /* server is shutting down */
    EBR_EUNSUPPORTED = -7  /* valid but not supported (e.g. a scan copy the index lacks) */
} ebr_status;

/* Arithmetic type of the ad-embedding scan. */
typedef enum { EBR_F32 = 0, EBR_BF16 = 1, EBR_FP8E4M3 = 2 } ebr_dtype;

typedef struct ebr_index ebr_index; /* opaque; immutable after build but for its launch shapes */

/* ------------------------------------------------------------------------ index */

/*
 * Index input, all host memory, copied during ebr_build_index.
 *  n_ads        N, 1 <= N < 2^32.
 *  dim          d, a multiple of 16 in [16, 128] (64 in the paper's towers,
 *               Section 4.1; wider with IPNN, Section 3.2).
 *  ad_emb       N x d FP32, row-major; the ground truth of the deep term.
 *  n_keys       V >= 0, number of posting lists (user feature values).
 *  key_offsets  V + 1 non-decreasing int64, key_offsets[0] == 0: key k owns
 *               postings [key_offsets[k], key_offsets[k+1]). Total < 2^32.
 *  post_ids     ad ids, strictly increasing within each key, < N (lists are
 *               sets, Algorithm 1 takes their union).
 *  post_w       FP32 cross weights per posting, or NULL for unit weights: the paper's
 *               binary L (Section 3.3, equation "hitmatch"; Algorithm 1 stores ids only),
 *               an ids-only index that stores and streams no weights.
 *  dtypes       bitmask of (1u << ebr_dtype) scan copies to build; FP32 is
 *               always built (it is also the exact rescore source). BF16 is
 *               round-to-nearest-even; FP8 is OCP e4m3fn with one FP32 scale per
 *               ad (max |e| / 448), round-to-nearest-even, saturating.
 * EBR_EINVAL: unsorted or duplicate postings, ids >= N, non-finite embeddings
 * or weights, d not a supported multiple of 16, totals out of range.
 */
typedef struct {
    int64_t n_ads;
    int32_t dim;
    const float* ad_emb;
    int64_t n_keys;
    const int64_t* key_offsets;
    const uint32_t* post_ids;
    const float* post_w;
    uint32_t dtypes;
} ebr_build_desc;

typedef struct {
    int64_t n_ads, n_keys, n_postings, n_chunks, n_tiles;
    int32_t dim, tile_ads;
    uint64_t arena_bytes;
    uint64_t bytes_emb_f32, bytes_emb_bf16, bytes_emb_fp8;
    uint64_t bytes_chunk_headers, bytes_packed_ids, bytes_weights;
    double max_err_bf16;     /* max over ads of ||e_a - bf16(e_a)||_2 (0 if not built) */
    double max_err_fp8;      /* max over ads of ||e_a - scale_a * fp8(e_a / scale_a)||_2 */
    double bits_per_id;      /* packed delta bits + header bits, per posting */
    double bytes_per_posting;/* whole posting store (headers + ids + weights) */
    double encode_ms;        /* host encode time of the last build */
    double upload_ms;        /* host-to-device copy time of the last build */
} ebr_index_info;

/* Exact arena size (bytes) ebr_build_index needs for desc: the storage of Section 3.4
 * ("Storage Layout", redesigned as in ebr_build_index) plus the embedding copies. Host only;
 * no GPU use. */
ebr_status ebr_index_size(const ebr_build_desc* desc, size_t* arena_bytes);

/*
 * Encode the posting lists (Section 3.4, "Block Compression" and "Storage
 * Layout", redesigned: 64-posting chunks of bit-packed id gaps with a per-key
 * chunk directory, raw FP32 weights), lay the embeddings out for the matrix
 * cores, and copy everything into dev_arena (device, >= ebr_index_size bytes,
 * 256-byte aligned). Synchronises hip_stream before returning. *out receives a
 * handle that owns host metadata only; free it with ebr_free_index.
 */
ebr_status ebr_build_index(const ebr_build_desc* desc, void* dev_arena, size_t arena_bytes,
                           void* hip_stream, ebr_index** out);

ebr_status ebr_index_stats(const ebr_index* index, ebr_index_info* out);

/* ------------------------------------------------------------------------ online refresh */

/*
 * Device-side build, for refreshing the index online: the paper rebuilds its GPU inverted
 * list whenever the feature-to-ad matrix is updated, every few minutes (Section 3.4), with a
 * parallel build of the lists (Algorithm 1; its preprocessing time is in Table 2). These
 * calls build the same index as ebr_build_index, arena byte for byte, with every step on the
 * GPU: list validation, chunk shapes and bit packing, per-key weight scales, the FP32 copy in
 * the matrix-core layout and the BF16 / FP8 copies. desc is as for ebr_build_index except
 * that its arrays (key_offsets, post_ids, post_w, ad_emb) are DEVICE pointers; only the
 * n_keys + 1 list offsets and a few counts travel to the host.
 *
 * scratch: device memory of ebr_device_build_scratch_size bytes (256-byte aligned), owned by
 * the caller, free again when the call returns. ebr_device_index_size gives the arena size
 * (as ebr_index_size does for host inputs); ebr_build_index_device fills dev_arena and
 * returns the handle (free it with ebr_free_index). Both synchronise hip_stream. Invalid
 * inputs (decreasing list offsets, ids not strictly increasing or >= n_ads, non-finite
 * weights or embeddings) give EBR_EINVAL, found on the GPU; the arena is then unspecified.
 */
ebr_status ebr_device_build_scratch_size(int64_t n_keys, int64_t n_postings, size_t* bytes);
ebr_status ebr_device_index_size(const ebr_build_desc* desc, void* scratch, size_t scratch_bytes,
                                 void* hip_stream, size_t* arena_bytes);
ebr_status ebr_build_index_device(const ebr_build_desc* desc, void* scratch, size_t scratch_bytes,
                                  void* dev_arena, size_t arena_bytes, void* hip_stream,
                                  ebr_index** out);

/*
 * Test hook: decode key's list on the GPU from the compressed arena (the inverse of the
 * encoding of Section 3.4, "Block Compression", as redesigned here) into the
 * device arrays ids / w of capacity cap; *len (host) receives the list length.
 * Blocking. EBR_ENOMEM if cap < length (nothing written).
 */
ebr_status ebr_decode_key(const ebr_index* index, int64_t key, uint32_t* ids, float* w,
                          int64_t cap, int64_t* len, void* hip_stream);

/*
 * Test hook: the same for the keys [key_begin, key_end), their lists concatenated in key
 * order (the layout of post_ids / post_w in ebr_build_desc, from key_offsets[key_begin]).
 * An index built without weights decodes them as 1. Blocking. EBR_EINVAL for a range
 * outside [0, V]; EBR_ENOMEM if cap is smaller than the postings (nothing written).
 */
ebr_status ebr_decode_keys(const ebr_index* index, int64_t key_begin, int64_t key_end, uint32_t* ids,
                           float* w, int64_t cap, int64_t* len, void* hip_stream);

void ebr_free_index(ebr_index* index);

/* ------------------------------------------------------------------------ query */

/*
 * One batch of queries.
 *  n_queries     B >= 0.
 *  user_emb      device, B x d FP32 row-major user vectors.
 *  feat_offsets  host, B + 1 int64 CSR over features, feat_offsets[0] == 0.
 *  feat_keys     host, keys of each query, distinct within a query, < V.
 *  feat_mult     host FP32 multiplier per feature (the paper's w_hat), or NULL
 *                for 1.0.
 *  k             host, per-query K, 0 <= K_q <= N. A query whose K_q (for reduced-precision
 *                scans rescore_factor * K_q) exceeds 8192, the selection path's in-LDS sort, is
 *                answered by a full sort of all N of its scores instead (FP32 scan, 64-bit
 *                cross-term cells; the workspace then holds 24 N bytes more): slower, same
 *                ordering rules.
 *  scan_dtype    EBR_F32: exact FP32 scan. EBR_BF16 / EBR_FP8E4M3: the scan streams that
 *                copy of the embeddings (EBR_EUNSUPPORTED if the index has none), keeps
 *                the rescore_factor * K_q best approximate candidates, rescores them
 *                exactly in FP32 and returns the top K_q; a per-query recall certificate
 *                (the K-th exact score exceeds every outsider's best possible exact score)
 *                is checked on the GPU, and a query that fails it is rerun with the FP32
 *                scan. The rescore computes each candidate's score with the FP32 scan's
 *                own arithmetic, so the results are the FP32 scan's ids and score bits.
 *  rescore_factor  candidates per result for reduced-precision scans (<= 0: 4). Ignored
 *                for F32.
 *  wide64        0: the cross term of Section 3.3 (equation "hitmatch") is summed in 32-bit
 *                fixed point with one quantum per query (2^-S, S the largest with
 *                sum_j |m_j| max|W[k_j,:]| 2^S below 2^31); a query whose worst-case
 *                rounding (F_q / 2 quanta) exceeds 2^-18 of the smallest returned score
 *                magnitude is rerun, inside the call, with 64-bit cells (quantum near
 *                2^-62 of that sum). 1: 64-bit cells for every query (FP32 scan only;
 *                EBR_EINVAL with BF16 / FP8). Results depend on the query alone either way.
 * Results of query q occupy positions [sum_{p<q} K_p, sum_{p<=q} K_p).
 */
typedef struct {
    int32_t n_queries;
    const float* user_emb;
    const int64_t* feat_offsets;
    const int32_t* feat_keys;
    const float* feat_mult;
    const int32_t* k;
    ebr_dtype scan_dtype;
    int32_t rescore_factor;
    int32_t wide64;
} ebr_batch;

/* Workspace bytes ebr_score_topk / ebr_score_dense need for this batch (its queries are the
 * inputs of Algorithm 2, Section 3.4). Host only. */
ebr_status ebr_workspace_size(const ebr_index* index, const ebr_batch* batch, size_t* bytes);

/*
 * Top-K of every query of the batch: for each query (its non-zero feature values
 * {(k, w_hat)}, the input of Algorithm 2 in Section 3.4, plus its user vector) the
 * score s(u, a) of every ad (the summed logits of Section 3.1; the cross term of
 * Section 3.3, equation "hitmatch") and the K ads with the largest scores (retrieval
 * keeps a high-scoring subset, Section 3.1; top-k retrieval, Section 2; ties go to the
 * smaller ad id, which the paper leaves open). ws: device workspace of ws_bytes >=
 * ebr_workspace_size (256-byte aligned). out_ids (uint32) and out_scores (FP32
 * s(u, a)) are device arrays of sum K_q entries, each query's slice ordered by
 * (score descending, id ascending); -0.0 scores are returned as +0.0.
 * The call blocks until the results are complete on hip_stream. The kernels run
 * in the launch shape recorded for the batch's dtype and query-group count
 * (ebr_autotune, ebr_set_launch_shape), else the default; results do not depend on it.
 * EBR_EINVAL: keys out of range or repeated in a query, K_q out of range,
 * non-finite multipliers or user vectors.
 */
ebr_status ebr_score_topk(const ebr_index* index, const ebr_batch* batch, void* ws,
                          size_t ws_bytes, uint32_t* out_ids, float* out_scores,
                          void* hip_stream);

/*
 * Test hook for small inventories: the full B x N FP32 deep and wide terms as
 * the top-K path computes them (row-major, device): the dual-tower inner product
 * (Section 3.1, equation "dual-tower") and the HitMatch cross term (Section 3.3,
 * equation "hitmatch"; the dense result of Algorithm 2 in Section 3.4). The path's score of ad a
 * for query q is exactly the FP32 sum deep[q*N+a] + wide[q*N+a]. Blocking.
 */
ebr_status ebr_score_dense(const ebr_index* index, const ebr_batch* batch, void* ws,
                           size_t ws_bytes, float* deep, float* wide, void* hip_stream);

/* ------------------------------------------------------------------------ no allocation */

/* Bytes of the device scratch behind ebr_score_topk_noalloc (256 MiB per GPU). */
#define EBR_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/*
 * For callers that cannot allocate device memory or hand over a workspace (work under HIP
 * stream capture, serving loops and harnesses that forbid hipMalloc): ebr_score_topk with
 * its workspace taken from a fixed array of EBR_NOALLOC_SCRATCH_BYTES bytes of device memory
 * inside the library, one per GPU, which exists while the library is loaded (for the life of
 * the process). Arguments as ebr_score_topk without the workspace; the results are identical
 * to ebr_score_topk's. The call allocates nothing: a batch whose workspace
 * (ebr_workspace_size) exceeds the array is refused with EBR_ENOMEM before any device work
 * (ebr_score_topk then serves it). Every call on one GPU uses that GPU's array, which keeps
 * the last call's contents (each call initialises what it reads): calls that overlap on one
 * GPU, from several threads or streams, race on it and must be serialised by the caller.
 */
ebr_status ebr_score_topk_noalloc(const ebr_index* index, const ebr_batch* batch,
                                  uint32_t* out_ids, float* out_scores, void* hip_stream);

/* ------------------------------------------------------------------------ launch shapes */

/*
 * How a batch's work is divided among work-groups. Section 3.4 (with Algorithm 2)
 * hands every thread an equal share of the posting work; here the shares are
 *  score_ranges   contiguous ranges of 32-ad tiles per query group in the candidate
 *                 scan: one work-group per (range, group); 0 = one work-group per
 *                 compute unit, ranges rounded down to a multiple of 8 (one range's
 *                 work-groups then share an XCD and its L2)
 *  sample_ranges  the same for the threshold pre-pass over the sample tiles
 *  decode_chunks  64-posting chunks one decode wavefront takes, 1..64 (0 = 8)
 * Any shape gives bit-identical results (the cross term is an exact fixed-point sum
 * and the outputs are sorted); only the time changes. Ranges are clamped to the
 * number of tiles; score_ranges * query groups must stay <= 2^24.
 */
typedef struct {
    int32_t score_ranges;
    int32_t sample_ranges;
    int32_t decode_chunks;
} ebr_launch_shape;

#define EBR_TUNE_MAX 16

/*
 * Autotuner report: the shapes tried, in order, with the median device time of the
 * whole batch (decode through rescore, HIP events on the call's stream) under each;
 * tried[0] is the default shape. best is the fastest; best_ms its time.
 */
typedef struct {
    int32_t n_tried;
    ebr_launch_shape tried[EBR_TUNE_MAX];
    float tried_ms[EBR_TUNE_MAX];
    ebr_launch_shape best;
    float best_ms;
    float default_ms;
} ebr_tune_report;

/*
 * Autotuner (launch tuning is this library's, not the paper's; the batch is the query input of
 * Algorithm 2, Section 3.4). Runs `batch` (as ebr_score_topk, same workspace and outputs) under the
 * default shape and then under candidate shapes, one field at a time (score ranges
 * at 1, 2 and 4 work-groups per compute unit; then sample ranges; then 4, 8, 16 and
 * 32 decode chunks per wavefront), `reps` timed runs each (<= 0: 3) after one
 * untimed run, keeping each field's fastest value. The winner is recorded in the
 * index for batches with the same scan dtype and the same number of query groups
 * (256 queries each at d <= 64, 128 above); ebr_score_topk, ebr_score_topk_graph and
 * the serving loop then use it. The outputs hold the batch's results on return.
 * The index's table is guarded by a mutex: tuning may overlap other calls.
 * Errors as ebr_score_topk; out may be NULL.
 */
ebr_status ebr_autotune(ebr_index* index, const ebr_batch* batch, void* ws, size_t ws_bytes,
                        uint32_t* out_ids, float* out_scores, int32_t reps, void* hip_stream,
                        ebr_tune_report* out);

/*
 * Set (shape non-NULL) or clear (NULL) the recorded shape for batches of n_queries
 * queries on scan_dtype, or read the shape such a batch would use (zero fields: the
 * default). EBR_EINVAL: n_queries < 1, an unknown dtype, fields out of range.
 */
ebr_status ebr_set_launch_shape(ebr_index* index, ebr_dtype scan_dtype, int32_t n_queries,
                                const ebr_launch_shape* shape);
ebr_status ebr_get_launch_shape(const ebr_index* index, ebr_dtype scan_dtype, int32_t n_queries,
                                ebr_launch_shape* out);

/* ------------------------------------------------------------------------ graphs */

/*
 * A batch's device work as one HIP graph. ebr_score_topk_graph plans the batch on
 * the host like ebr_score_topk and copies the plan to the device on hip_stream (from
 * the handle's pinned staging); it records the batch's kernel sequence (decode,
 * pre-pass, the gated selection rounds, and for reduced-precision scans the exact
 * rescore) by stream capture on the handle's own stream, loads it into the handle's
 * executable graph (an in-place update when the sequence has the same nodes as the
 * last one, else a new instantiation) and launches that on hip_stream. What follows the graph is as in ebr_score_topk and
 * rare: extra selection rounds, and the FP32 rerun of queries whose recall
 * certificate failed. Results are bit-identical to ebr_score_topk's.
 * The handle owns a HIP stream of the device current at create (default priority),
 * the executable graph and pinned host staging that grows to the largest plan seen
 * (hipHostMalloc); it allocates no device memory. A handle serves one call at a
 * time (calls block until their results are complete, so consecutive calls on one
 * thread are fine); give each thread its own. Per-phase timings are not recorded
 * for graph calls.
 */
typedef struct ebr_graph ebr_graph; /* opaque */

typedef struct {
    uint64_t calls;           /* ebr_score_topk_graph calls that launched a graph */
    uint64_t instantiations;  /* new executable graphs */
    uint64_t updates;         /* in-place updates of the executable graph */
    uint64_t nodes;           /* nodes of the last recorded sequence */
} ebr_graph_info;

ebr_status ebr_graph_create(ebr_graph** out);
ebr_status ebr_score_topk_graph(ebr_graph* graph, const ebr_index* index, const ebr_batch* batch,
                                void* ws, size_t ws_bytes, uint32_t* out_ids, float* out_scores,
                                void* hip_stream);
ebr_status ebr_graph_stats(const ebr_graph* graph, ebr_graph_info* out);
void ebr_graph_destroy(ebr_graph* graph);

/* ------------------------------------------------------------------------ timing */

/*
 * Per-phase device times of the last ebr_score_topk on the calling thread,
 * measured with HIP events recorded on the call's stream around each phase
 * (only while timing is enabled with ebr_set_timing(1); off by default).
 *  decode_ms    batch key dedup upload, posting decode into tile buckets
 *  sample_ms    scoring of the sample tiles and the per-query threshold select
 *  score_ms     the fused scoring kernel over the whole inventory (all rounds)
 *  finalize_ms  candidate sort and output (all rounds)
 *  host_ms      host validation and planning
 *  score_first_ms  the fused scoring kernel of the first round alone
 *  rescore_ms   exact FP32 rescore of the candidates (reduced-precision scans)
 *  rounds       scoring rounds (1 unless a threshold had to be revised)
 *  uncertified  queries of a reduced-precision scan whose recall certificate failed and
 *               that were therefore rerun with the FP32 scan
 *  imprecise    queries rerun with 64-bit cross-term cells (see ebr_batch.wide64)
 */
typedef struct {
    double decode_ms, sample_ms, score_ms, finalize_ms, host_ms, score_first_ms, rescore_ms;
    int32_t rounds, uncertified, imprecise;
} ebr_timings;

ebr_status ebr_set_timing(int enable);
ebr_status ebr_get_timings(ebr_timings* out);

/* ------------------------------------------------------------------------ serving */

/*
 * Serving loop over a resident index. Retrieval answers user requests one at a
 * time under throughput and latency demands (Section 2 on the retrieval stage;
 * Section 4.1 takes maximum QPS as an efficiency metric; Section 4.4 runs the
 * operator online over millions of ads); the GPU is efficient only on batches. A server accepts single queries from any thread (ebr_submit), groups
 * whatever has arrived into batches under a scratch budget, and keeps up to
 * `pipeline` batches in flight on as many HIP streams, so that queries arriving
 * while a batch runs are admitted into the next one without waiting for it
 * (continuous batching at batch granularity). Every batch runs the same path
 * as ebr_score_topk, so a query's results are bit-identical whatever batch it
 * lands in.
 *
 * Scratch: a caller-owned device arena of scratch_bytes (256-byte aligned),
 * split evenly between the pipeline slots. A slot holds one batch's user rows,
 * outputs and workspace; a batch admits queued queries first-in first-out
 * while the workspace of the batch so far (computed exactly from its sizes:
 * distinct keys, their postings, queries, K) fits the slot.
 * The library allocates pinned host staging (hipHostMalloc) and streams at
 * create and frees them at destroy; it allocates no device memory.
 */
typedef struct ebr_server ebr_server; /* opaque */

/*
 *  max_batch     queries per batch, 1..4096 (0: 256)
 *  max_wait_us   how long the oldest queued query may wait for a fuller batch
 *                before its batch is launched (0: launch at once with what is
 *                queued; < 0: 0)
 *  pipeline      batches in flight, 1..4 (0: 2)
 *  scan_dtype, rescore_factor   as in ebr_batch, for every query
 *  graph         nonzero: each slot runs its batches through its own ebr_graph
 *                handle (ebr_score_topk_graph) instead of launching them eagerly
 *  f32_below     batches of at most this many queries run the FP32 scan whatever
 *                scan_dtype says (0: never). The FP32 scan has a faster path for
 *                groups of at most 16 queries, and the exact rescore of the reduced-
 *                precision scans returns the FP32 scan's ids and score bits, so a
 *                query's results do not depend on which scan its batch took.
 *  max_queue     most queries waiting for a batch (not yet on the GPU); ebr_submit
 *                returns EBR_EAGAIN while the queue is that full (0: 16 x max_batch)
 * Batches use the launch shape recorded in the index (ebr_autotune) for their
 * dtype and query-group count.
 *
 * Fault injection (tests of the error path): if the environment variable
 * EBR_FAULT_BATCH holds a number n >= 0 when the server is created, the server's
 * batch number n (counted from 0) reports EBR_EDEVICE to every ticket it holds
 * instead of writing results; the batches before and after it run normally.
 */
typedef struct {
    int32_t max_batch;
    int32_t max_wait_us;
    int32_t pipeline;
    ebr_dtype scan_dtype;
    int32_t rescore_factor;
    int32_t graph;
    int32_t f32_below;
    int32_t max_queue;
} ebr_server_opts;

/*
 * One query, all host memory, copied by ebr_submit:
 *  user_emb   d FP32 values (finite)
 *  n_feats    number of features (>= 0)
 *  feat_keys  n_feats distinct keys < n_keys
 *  feat_mult  n_feats finite multipliers, or NULL (all 1)
 *  k          0 <= k <= min(n_ads, 8192 / f), f = 1 for F32, else the rescore factor
 */
typedef struct {
    const float* user_emb;
    int32_t n_feats;
    const int32_t* feat_keys;
    const float* feat_mult;
    int32_t k;
} ebr_query;

/*
 * Latency is per query, from ebr_submit to the moment its results are written
 * to the caller's buffers (host steady clock); percentiles over every query
 * completed since create or the last ebr_server_reset_stats.
 *  submitted, completed, failed   query counts; queued: waiting for a batch now;
 *  rejected       submissions refused with EBR_EAGAIN because the queue was full
 *  batches        batches launched; mean_batch: queries per batch
 *  p50_ms, p99_ms, max_ms, mean_ms   latency
 *  elapsed_ms     wall time since create or reset; qps = completed / elapsed
 *  busy_ms        summed wall time of batches in flight (over slots)
 */
typedef struct {
    uint64_t submitted, completed, failed, queued, batches, rejected;
    double mean_batch, p50_ms, p99_ms, max_ms, mean_ms, elapsed_ms, qps, busy_ms;
} ebr_server_info;

/*
 * Start a server on the device current at the call (it must be the index's).
 * EBR_ENOMEM if one slot cannot hold a batch of one query with K = 1;
 * EBR_EUNSUPPORTED if the index holds no copy of scan_dtype.
 */
ebr_status ebr_server_create(const ebr_index* index, void* scratch, size_t scratch_bytes,
                             const ebr_server_opts* opts, ebr_server** out);

/*
 * Queue one query: its feature values {(k, w_hat)} (the input of Algorithm 2, Section 3.4),
 * its user vector and K (top-k retrieval, Section 2). ids_out (uint32) and scores_out (FP32) are host arrays of
 * q->k entries that must stay valid until ebr_poll reports the ticket done;
 * they are written in (score descending, id ascending) order. *ticket
 * identifies the query for ebr_poll. Thread-safe.
 * EBR_EINVAL for an invalid query; EBR_ENOMEM if the query alone does not fit
 * a slot; EBR_EAGAIN if max_queue queries are already waiting (nothing is
 * queued: poll some tickets, then submit again); EBR_ESHUTDOWN once destroy has begun.
 */
ebr_status ebr_submit(ebr_server* server, const ebr_query* q, uint32_t* ids_out,
                      float* scores_out, uint64_t* ticket);

/*
 * Wait up to timeout_us (< 0: without limit, 0: just look) for a ticket (its top-K, as
 * ebr_score_topk returns it; Section 3.1 and equation "hitmatch", Section 3.3).
 * EBR_OK: results written, the ticket is retired. EBR_EAGAIN: not done yet.
 * A failed batch reports its error (the ticket is retired).
 * EBR_ENOTFOUND: unknown or already retired ticket. Thread-safe.
 */
ebr_status ebr_poll(ebr_server* server, uint64_t ticket, int32_t timeout_us);

ebr_status ebr_server_stats(ebr_server* server, ebr_server_info* out);
ebr_status ebr_server_reset_stats(ebr_server* server);

/*
 * Online refresh of a serving loop (the paper refreshes the index while serving, Section
 * 3.4): queries submitted after this call run on `next`; each query submitted before it runs
 * on the index it was submitted to (a batch never mixes indexes). Returns once every query of
 * the previous index has completed (its results are in the caller's buffers, polled or not),
 * so the caller may then free that index and its arena; `next` must stay alive while the
 * server uses it. next must have the same ads and width as the current index and hold the
 * server's scan copy (EBR_EINVAL / EBR_EUNSUPPORTED otherwise); EBR_EAGAIN while another
 * swap is waiting. Thread-safe with submit and poll; blocks the calling thread.
 */
ebr_status ebr_server_swap_index(ebr_server* server, const ebr_index* next);

/*
 * Stop accepting queries, finish every queued and running one, release the
 * server's host resources. Results of tickets never polled are still written.
 */
ebr_status ebr_server_destroy(ebr_server* server);

/* ------------------------------------------------------------------------ codec */

/*
 * Host codec of one posting list in the index's chunk format (the lossless list compression
 * of Section 3.4, "Block Compression", redesigned for 64-wide wavefronts), for tests and
 * tools that have no GPU. ids: n strictly increasing uint32. The encoding is
 * ceil(n / 64) 16-byte chunk headers followed by the packed gap words.
 * ebr_codec_size: bytes ebr_codec_encode writes.
 * ebr_codec_decode: inverse; EBR_EINVAL on a malformed encoding.
 */
ebr_status ebr_codec_size(const uint32_t* ids, int64_t n, size_t* bytes);
ebr_status ebr_codec_encode(const uint32_t* ids, int64_t n, void* out, size_t cap,
                            size_t* used);
ebr_status ebr_codec_decode(const void* in, size_t bytes, int64_t n, uint32_t* ids);

/* ------------------------------------------------------------------------ quantisers */

/*
 * Host reference of the index's reduced-precision encodings, for tests (the paper studies no
 * reduced precision; the copies serve the approximate scan before the exact FP32 rescore of
 * the K' best, see ebr_batch.scan_dtype). BF16: round to
 * nearest even. FP8: OCP e4m3fn of in[i] / scale, round to nearest even, saturating at
 * +-448; ebr_dequantize_fp8 decodes codes to FP32 (without the scale).
 */
ebr_status ebr_quantize_bf16(const float* in, int64_t n, uint16_t* out);
ebr_status ebr_quantize_fp8(const float* in, int64_t n, float scale, uint8_t* out);
ebr_status ebr_dequantize_fp8(const uint8_t* in, int64_t n, float* out);

/* Thread-local text of the last error (never NULL). */
const char* ebr_last_error(void);

/* Library version string. */
const char* ebr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* EBR_H */
