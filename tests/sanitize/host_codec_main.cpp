// Sanitizer driver for the library's host-side codec and quantisers (built with
// -fsanitize=address,undefined by tests/test_sanitizers.py). Exits 0 when every
// round trip holds; any sanitizer report aborts with a non-zero status.
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "internal.h"

// The library keeps its error text in the runtime (api.cpp, which needs HIP); the driver
// links the host-only sources and keeps the last message itself.
namespace ebr {
static char g_msg[256];
void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
}
}  // namespace ebr

static uint64_t g_state = 0x9e3779b97f4a7c15ull;
static uint32_t next_u32() {  // splitmix64
    uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return (uint32_t)((z ^ (z >> 31)) >> 32);
}

static bool round_trip(const std::vector<uint32_t>& ids) {
    const int64_t n = (int64_t)ids.size();
    int64_t chunks = 0, words = 0;
    ebr::codec_measure(ids.data(), n, &chunks, &words);
    std::vector<ebr::ChunkHdr> hdr((size_t)chunks + 1);
    std::vector<uint32_t> w((size_t)words + 1);
    ebr::codec_encode(ids.data(), n, hdr.data(), w.data(), 0u, 0u);
    std::vector<uint32_t> back((size_t)n + 1);
    if (!ebr::codec_decode(hdr.data(), chunks, w.data(), words, n, back.data())) return false;
    return n == 0 || std::memcmp(back.data(), ids.data(), 4 * (size_t)n) == 0;
}

int main() {
    int bad = 0;
    const int64_t lengths[] = {0, 1, 2, 63, 64, 65, 127, 128, 129, 1000, 5000};
    for (int64_t len : lengths) {
        // random strictly increasing ids with random gaps, consecutive ids, maximal gaps
        for (int kind = 0; kind < 3; ++kind) {
            std::vector<uint32_t> ids;
            uint64_t v = kind == 2 ? 0 : next_u32() % 1000;
            for (int64_t i = 0; i < len; ++i) {
                ids.push_back((uint32_t)v);
                const uint64_t gap = kind == 0 ? 1 + next_u32() % 5000 : kind == 1 ? 1 : 0xffffffffull / (uint64_t)(len + 1);
                v += gap;
                if (v > 0xffffffffull) break;
            }
            if (!round_trip(ids)) { std::printf("codec round trip failed: length %lld kind %d\n", (long long)len, kind); ++bad; }
        }
    }
    // ids at both ends of the range
    if (!round_trip({0u, 1u, 0xfffffffeu, 0xffffffffu})) { std::printf("codec extremes failed\n"); ++bad; }
    // FP8 codes: every finite code survives decode then encode; BF16 keeps exact values
    for (int c = 0; c < 256; ++c) {
        if ((c & 0x7f) == 0x7f) continue;  // NaN codes
        const float x = ebr::fp8_e4m3_to_f32((uint8_t)c);
        const uint8_t back = ebr::fp8_e4m3_rne(x);
        if (back != (uint8_t)c && !(x == 0.0f && (back & 0x7f) == 0)) { std::printf("fp8 code %d -> %d\n", c, back); ++bad; }
    }
    const float specials[] = {0.0f, -0.0f, 1.0f, -2.5f, std::numeric_limits<float>::denorm_min(),
                              std::numeric_limits<float>::min(), std::numeric_limits<float>::max(),
                              -std::numeric_limits<float>::max(), 448.0f, 1e-9f, 3.0e38f};
    for (float x : specials) {
        const uint16_t h = ebr::bf16_rne(x);
        const float y = ebr::bf16_to_f32(h);
        // half a BF16 unit in the last place: 2^-8 relative, 2^-134 among subnormals
        const float tol = std::fmax(std::fabs(x) * (1.0f / 256.0f), std::ldexp(1.0f, -134));
        if (std::isfinite(y) && std::fabs(y - x) > tol) { std::printf("bf16 %g -> %g\n", x, y); ++bad; }
        (void)ebr::fp8_e4m3_rne(x);
    }
    std::vector<float> in(1000);
    for (float& x : in) x = (float)((int32_t)next_u32()) * 1e-9f;
    std::vector<uint16_t> hb(in.size());
    std::vector<uint8_t> f8(in.size());
    std::vector<float> back(in.size());
    if (ebr_quantize_bf16(in.data(), (int64_t)in.size(), hb.data()) != EBR_OK) ++bad;
    if (ebr_quantize_fp8(in.data(), (int64_t)in.size(), 1.0f, f8.data()) != EBR_OK) ++bad;
    if (ebr_dequantize_fp8(f8.data(), (int64_t)f8.size(), back.data()) != EBR_OK) ++bad;
    std::printf("%s\n", bad ? "FAILED" : "ok");
    return bad ? 1 : 0;
}
