// FP64 CPU oracle for Wide & Deep ad retrieval (arXiv 2511.22460).
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call
// this file; only the test suite, the smoke check and the CPU-baseline leg of
// the benchmark do. It shares no code with the GPU library: it reads the raw
// inputs (FP32 embeddings, uncompressed posting lists) exactly as they are
// handed to the library's index build and batch calls.
//
// What it computes, per query q and ad a, all in FP64:
//   deep(a) = sum_i u_q[i] * E[a][i]
//       The dual-tower inner product (Section 3.1, equation "dual-tower"); with
//       IPNN the two vectors are just longer (Section 3.2, the concatenated
//       logit), so d is a parameter. A product of two FP32 values is exact in
//       FP64, so the only rounding is in the d-term sum.
//   wide(a) = sum over query features j, and over postings t of key k_j with
//             id P_k[t] == a, of m_j * W_k[t]
//       The HitMatch cross term (Section 3.3, equation "hitmatch"): the paper's
//       binary L with per-feature weight w_i x_i is the special case W == 1,
//       m_j = w_j x_j; Section 3.4 writes the same sum as the product L * w~.
//   s(a)    = deep(a) + wide(a)
//       The logits are summed (Section 3.1, caption of the model figure).
//   cond(a) = sum_i |u_q[i] E[a][i]| + sum |m_j W_k[t]|
//       A condition magnitude used only to judge cancellation in tests.
// Top-K: ads ordered by (s descending, id ascending), the first K kept. The
// paper asks for the top-k high-scoring ads (Sections 2 and 3.1) and fixes no
// tie rule; ties go to the smaller ad id.
//
// Build: g++ -O2 -std=c++17 -fopenmp -fPIC -shared oracle.cpp -o liboracle.so
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <omp.h>
#include <vector>

extern "C" {

// Per-ad FP64 deep, wide and cond terms of one query. Any output may be null.
// Returns 0, or -1 on an out-of-range key or posting id.
int oracle_scores(int64_t n_ads, int32_t dim, const float* ad_emb,
                  int64_t n_keys, const int64_t* key_offsets, const uint32_t* post_ids,
                  const float* post_w,
                  const float* u, int32_t n_feat, const int32_t* keys, const float* mult,
                  double* deep, double* wide, double* cond) {
    // deep term and its magnitude: one independent dot product per ad
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < n_ads; ++a) {
        const float* e = ad_emb + a * dim;
        double s = 0.0, c = 0.0;
        for (int32_t i = 0; i < dim; ++i) {
            double p = (double)u[i] * (double)e[i];
            s += p;
            c += std::fabs(p);
        }
        if (deep) deep[a] = s;
        if (cond) cond[a] = c;
    }
    if (wide) std::fill(wide, wide + n_ads, 0.0);
    // wide term: walk each feature's posting list and add m * w at each listed ad
    for (int32_t j = 0; j < n_feat; ++j) {
        int64_t k = keys[j];
        if (k < 0 || k >= n_keys) return -1;
        double m = mult ? (double)mult[j] : 1.0;
        for (int64_t t = key_offsets[k]; t < key_offsets[k + 1]; ++t) {
            int64_t a = post_ids[t];
            if (a >= n_ads) return -1;
            double v = m * (double)post_w[t];
            if (wide) wide[a] += v;
            if (cond) cond[a] += std::fabs(v);
        }
    }
    return 0;
}

// Top-K of one query: ids, FP64 scores and cond, ordered by (score desc, id asc).
// deep_out / wide_out (nullable) receive the two terms of each returned ad.
int oracle_topk(int64_t n_ads, int32_t dim, const float* ad_emb,
                int64_t n_keys, const int64_t* key_offsets, const uint32_t* post_ids,
                const float* post_w,
                const float* u, int32_t n_feat, const int32_t* keys, const float* mult,
                int64_t k, uint32_t* out_ids, double* out_scores, double* out_cond,
                double* deep_out, double* wide_out) {
    if (k < 0 || k > n_ads) return -1;
    std::vector<double> deep(n_ads), wide(n_ads), cond(n_ads), s(n_ads);
    int rc = oracle_scores(n_ads, dim, ad_emb, n_keys, key_offsets, post_ids, post_w,
                           u, n_feat, keys, mult, deep.data(), wide.data(), cond.data());
    if (rc) return rc;
    for (int64_t a = 0; a < n_ads; ++a) s[a] = deep[a] + wide[a];
    std::vector<int64_t> order(n_ads);
    std::iota(order.begin(), order.end(), (int64_t)0);
    auto before = [&](int64_t x, int64_t y) {
        if (s[x] != s[y]) return s[x] > s[y];
        return x < y;
    };
    std::partial_sort(order.begin(), order.begin() + k, order.end(), before);
    for (int64_t i = 0; i < k; ++i) {
        int64_t a = order[i];
        out_ids[i] = (uint32_t)a;
        if (out_scores) out_scores[i] = s[a];
        if (out_cond) out_cond[i] = cond[a];
        if (deep_out) deep_out[i] = deep[a];
        if (wide_out) wide_out[i] = wide[a];
    }
    return 0;
}

// The same for a batch: query q's results start at out_offsets[q] (= sum of the earlier K
// values); feat_offsets has B + 1 entries. Queries are independent, so they are spread over
// the OpenMP threads (each query's own loops then run on its one thread); a batch smaller
// than the thread count runs its queries one after another, each over all threads. Returns
// 0, or the first error code of any query.
int oracle_topk_batch(int64_t n_ads, int32_t dim, const float* ad_emb,
                      int64_t n_keys, const int64_t* key_offsets, const uint32_t* post_ids,
                      const float* post_w,
                      int32_t n_queries, const float* user_emb, const int64_t* feat_offsets,
                      const int32_t* feat_keys, const float* feat_mult, const int32_t* kq,
                      const int64_t* out_offsets, uint32_t* out_ids, double* out_scores,
                      double* out_cond) {
    int rc_all = 0;
    const bool across = n_queries >= omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) if (across)
    for (int32_t q = 0; q < n_queries; ++q) {
        int64_t f0 = feat_offsets[q], f1 = feat_offsets[q + 1];
        int64_t o = out_offsets[q];
        int rc = oracle_topk(n_ads, dim, ad_emb, n_keys, key_offsets, post_ids, post_w,
                             user_emb + (int64_t)q * dim, (int32_t)(f1 - f0), feat_keys + f0,
                             feat_mult ? feat_mult + f0 : nullptr, kq[q], out_ids + o,
                             out_scores ? out_scores + o : nullptr,
                             out_cond ? out_cond + o : nullptr, nullptr, nullptr);
        if (rc) {
#pragma omp critical
            if (!rc_all) rc_all = rc;
        }
    }
    return rc_all;
}

int oracle_num_threads(void) {
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}

}  // extern "C"
