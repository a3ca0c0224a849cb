// Sanitizer driver for the FP64 oracle (built with -fsanitize=address,undefined by
// tests/test_sanitizers.py): a small random inventory, several queries and K values,
// and the order, distinctness and score checks of every result. Exits 0 when they hold.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <set>
#include <vector>

extern "C" int oracle_topk(int64_t n_ads, int32_t dim, const float* ad_emb, int64_t n_keys,
                           const int64_t* key_offsets, const uint32_t* post_ids, const float* post_w,
                           const float* u, int32_t n_feat, const int32_t* keys, const float* mult,
                           int64_t k, uint32_t* out_ids, double* out_scores, double* out_cond,
                           double* deep_out, double* wide_out);

static uint64_t g_state = 12345;
static double uniform() {  // splitmix64 -> [0, 1)
    uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return (double)((z ^ (z >> 31)) >> 11) * 0x1.0p-53;
}

int main() {
    const int64_t N = 3001, V = 40;
    const int32_t d = 16;
    std::vector<float> E((size_t)N * d);
    for (float& x : E) x = (float)(uniform() - 0.5);
    std::vector<int64_t> off(V + 1, 0);
    std::vector<uint32_t> ids;
    std::vector<float> w;
    for (int64_t k = 0; k < V; ++k) {
        for (int64_t a = 0; a < N; ++a)
            if (uniform() < 0.05 * (double)(k % 4)) { ids.push_back((uint32_t)a); w.push_back((float)(uniform() - 0.5)); }
        off[k + 1] = (int64_t)ids.size();
    }
    int bad = 0;
    for (int q = 0; q < 6; ++q) {
        std::vector<float> u(d);
        for (float& x : u) x = q == 5 ? 0.0f : (float)(uniform() - 0.5);  // q = 5: heavy ties
        std::vector<int32_t> keys;
        std::vector<float> mult;
        for (int32_t k = 0; k < V; k += 3 + q) { keys.push_back(k); mult.push_back(q == 5 ? 1.0f : (float)uniform()); }
        for (int64_t K : {(int64_t)0, (int64_t)1, (int64_t)100, N}) {
            std::vector<uint32_t> out((size_t)K + 1);
            std::vector<double> sc((size_t)K + 1), cond((size_t)K + 1), dp((size_t)K + 1), wd((size_t)K + 1);
            if (oracle_topk(N, d, E.data(), V, off.data(), ids.data(), w.data(), u.data(),
                            (int32_t)keys.size(), keys.data(), mult.data(), K, out.data(), sc.data(),
                            cond.data(), dp.data(), wd.data()) != 0) { ++bad; continue; }
            std::set<uint32_t> seen;
            for (int64_t i = 0; i < K; ++i) {
                seen.insert(out[i]);
                if (sc[i] != dp[i] + wd[i] || cond[i] < std::fabs(sc[i])) ++bad;
                if (i > 0 && (sc[i] > sc[i - 1] || (sc[i] == sc[i - 1] && out[i] < out[i - 1]))) ++bad;
            }
            if ((int64_t)seen.size() != K) ++bad;
        }
    }
    // out-of-range key: an error, not a crash
    std::vector<float> u(d, 0.5f);
    int32_t badkey = (int32_t)V;
    uint32_t o1;
    double s1;
    if (oracle_topk(N, d, E.data(), V, off.data(), ids.data(), w.data(), u.data(), 1, &badkey, nullptr, 1,
                    &o1, &s1, nullptr, nullptr, nullptr) == 0) ++bad;
    std::printf("%s\n", bad ? "FAILED" : "ok");
    return bad ? 1 : 0;
}
