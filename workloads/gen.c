/*
 * Seeded synthetic inputs shaped like the paper's ad-retrieval workloads.
 *
 * This file generates inputs only. It holds none of the scoring, ranking or
 * index arithmetic of the method: both the FP64 oracle and the GPU library
 * consume what it writes, and neither shares any other code.
 *
 * Random numbers come from a counter-based generator: draw(key, ctr) is the
 * SplitMix64 output function (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) applied to key + ctr * gamma,
 * with gamma = 0x9E3779B97F4A7C15. Every array element is a pure function of
 * (seed, stream, index), so the output does not depend on the thread count.
 *
 * Exported (C ABI, all host memory, caller-allocated outputs):
 *   wl_normal_rows  - n rows of d N(0,1) values, each row L2-normalised (FP64
 *                     norm), stored FP32.
 *   wl_lists        - per key k an exact-length, strictly increasing,
 *                     uniformly random subset of [0, n_ads) plus N(0, sigma)
 *                     FP32 weights.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t draw(uint64_t key, uint64_t ctr) { return mix64(key + ctr * GAMMA); }
/* uniform in the open interval (0, 1) */
static inline double unit_open(uint64_t x) { return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
static inline uint64_t stream_key(uint64_t seed, uint64_t tag) { return mix64(mix64(seed) ^ mix64(tag * GAMMA + 1)); }

/* Box-Muller: element j of a stream uses the pair (2*(j/2), 2*(j/2)+1); even j takes the cosine, odd j the sine. */
static inline double normal_at(uint64_t key, uint64_t j) {
    uint64_t p = j >> 1;
    double u1 = unit_open(draw(key, 2 * p));
    double u2 = unit_open(draw(key, 2 * p + 1));
    double r = sqrt(-2.0 * log(u1));
    double t = 6.283185307179586476925 * u2;
    return (j & 1) ? r * sin(t) : r * cos(t);
}

void wl_normal_rows(uint64_t seed, uint64_t tag, int64_t n, int32_t d, float* out) {
    uint64_t key = stream_key(seed, tag);
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < n; ++a) {
        double buf[1024];
        double ss = 0.0;
        for (int32_t i = 0; i < d; ++i) {
            double v = normal_at(key, (uint64_t)a * (uint64_t)d + (uint64_t)i);
            buf[i & 1023] = v;
            ss += v * v;
        }
        double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
        for (int32_t i = 0; i < d; ++i) out[a * d + i] = (float)(buf[i & 1023] * inv);
    }
}

/*
 * One list: an exact-size uniform subset of [0, n_ads), sorted.
 * Draw a Bernoulli(p) subset by geometric gaps with p a little above
 * len / n_ads, retrying with a larger p until it holds at least len ids, then
 * drop cnt - len of them chosen uniformly (Floyd's sampling of distinct
 * indices). A uniform len-subset of a uniform random subset is a uniform
 * len-subset, and dropping keeps the ids sorted.
 */
static int one_list(uint64_t key, int64_t len, int64_t n_ads, uint32_t* ids_out) {
    if (len <= 0) return 0;
    double p = ((double)len + 4.0 * sqrt((double)len) + 16.0) / (double)n_ads;
    int64_t cap = 0;
    uint32_t* tmp = NULL;
    for (uint64_t attempt = 0;; ++attempt) {
        if (p > 1.0) p = 1.0;
        int64_t want = (p >= 1.0) ? n_ads : (int64_t)((double)n_ads * p + 8.0 * sqrt((double)n_ads * p) + 64.0);
        if (want > n_ads) want = n_ads;
        if (want > cap) {
            free(tmp);
            cap = want;
            tmp = (uint32_t*)malloc((size_t)cap * sizeof(uint32_t));
            if (!tmp) return -1;
        }
        int64_t cnt = 0;
        uint64_t ctr = attempt << 40;
        if (p >= 1.0) {
            for (int64_t a = 0; a < n_ads; ++a) tmp[cnt++] = (uint32_t)a;
        } else {
            double lq = log1p(-p);
            int64_t cur = -1;
            for (;;) {
                double u = unit_open(draw(key, ctr++));
                double g = floor(log(u) / lq);
                if (g > (double)n_ads) break;
                cur += 1 + (int64_t)g;
                if (cur >= n_ads) break;
                if (cnt == cap) {
                    cap = cap * 2;
                    uint32_t* t2 = (uint32_t*)realloc(tmp, (size_t)cap * sizeof(uint32_t));
                    if (!t2) { free(tmp); return -1; }
                    tmp = t2;
                }
                tmp[cnt++] = (uint32_t)cur;
            }
        }
        if (cnt >= len) {
            int64_t drop = cnt - len;
            uint8_t* gone = (uint8_t*)calloc((size_t)cnt, 1);
            if (!gone) { free(tmp); return -1; }
            uint64_t tk = mix64(key ^ 0x5bd1e995ULL);
            uint64_t c2 = attempt << 40;
            for (int64_t j = cnt - drop; j < cnt; ++j) {
                int64_t t = (int64_t)(draw(tk, c2++) % (uint64_t)(j + 1));
                if (gone[t]) gone[j] = 1; else gone[t] = 1;
            }
            int64_t o = 0;
            for (int64_t i = 0; i < cnt; ++i)
                if (!gone[i]) ids_out[o++] = tmp[i];
            free(gone);
            free(tmp);
            return 0;
        }
        p = p * 1.25 + 1e-9;
    }
}

/*
 * offsets: n_keys + 1 prefix sums of lengths (offsets[0] == 0), supplied by
 * the caller. Returns 0, or -1 if a length exceeds n_ads or memory runs out.
 */
int wl_lists(uint64_t seed, int64_t n_keys, const int64_t* offsets, int64_t n_ads,
             double w_sigma, uint32_t* ids, float* w) {
    int bad = 0;
    uint64_t base_ids = stream_key(seed, 0x1d5);
    uint64_t base_w = stream_key(seed, 0x3e7);
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
    for (int64_t k = 0; k < n_keys; ++k) {
        int64_t len = offsets[k + 1] - offsets[k];
        if (len > n_ads) { bad |= 1; continue; }
        uint64_t kid = mix64(base_ids + (uint64_t)k * GAMMA);
        if (one_list(kid, len, n_ads, ids + offsets[k]) != 0) { bad |= 1; continue; }
        uint64_t kw = mix64(base_w + (uint64_t)k * GAMMA);
        for (int64_t t = 0; t < len; ++t) w[offsets[k] + t] = (float)(w_sigma * normal_at(kw, (uint64_t)t));
    }
    return bad ? -1 : 0;
}
