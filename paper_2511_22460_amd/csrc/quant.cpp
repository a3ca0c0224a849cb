// Reduced-precision copies of the ad embeddings (host side, at index build).
//
// BF16: round-to-nearest-even from FP32 (the top 16 bits of the FP32 pattern after adding
// 0x7fff plus the lowest kept bit).
// FP8: OCP e4m3fn (1 sign, 4 exponent bits with bias 7, 3 mantissa bits; no infinities;
// largest finite 448; subnormals m * 2^-9) with one FP32 scale per ad row,
// scale = max_i |e_i| / 448; codes are round-to-nearest-even of e_i / scale, saturating.
// Both copies are laid out for v_mfma_f32_32x32x16_bf16 (see k_score in score.h).
#include <cmath>
#include <cstring>

#include "internal.h"

namespace ebr {

uint16_t bf16_rne(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    const uint32_t bias = 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)((u + bias) >> 16);
}

float bf16_to_f32(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// e4m3fn encode with round-to-nearest-even and saturation to +-448. x must be finite.
uint8_t fp8_e4m3_rne(float x) {
    const uint8_t sign = std::signbit(x) ? 0x80 : 0x00;
    double a = std::fabs((double)x);
    if (a >= 448.0) return sign | 0x7e;
    if (a < std::ldexp(1.0, -6)) {  // subnormal range: multiples of 2^-9
        const double m = std::nearbyint(std::ldexp(a, 9));  // default mode: ties to even
        return sign | (uint8_t)m;                            // m == 8 is the smallest normal
    }
    int e;
    const double f = std::frexp(a, &e);  // a = f * 2^e, f in [0.5, 1)
    int ex = e - 1;                      // a = (2 f) * 2^ex, 2 f in [1, 2)
    double m = std::nearbyint((2.0 * f - 1.0) * 8.0);
    if (m >= 8.0) { m = 0.0; ++ex; }
    if (ex > 8 || (ex == 8 && m > 6.0)) return sign | 0x7e;
    return sign | (uint8_t)(((ex + 7) << 3) | (int)m);
}

float fp8_e4m3_to_f32(uint8_t c) {
    const int s = c >> 7, e = (c >> 3) & 15, m = c & 7;
    if (e == 15 && m == 7) return std::nanf("");
    const double v = e == 0 ? std::ldexp((double)m, -9) : std::ldexp(1.0 + m / 8.0, e - 7);
    return (float)(s ? -v : v);
}

// Element (row a, dim k) of the 32x32x16 BF16 B-operand layout: per 32-ad block b, per
// 16-dim step s, 64 lanes x 8 values; lane l, value j holds e[32b + (l & 31)][16s + 8(l >> 5) + j].
size_t mfma16_index(int64_t a, int k, int d) {
    const int64_t b = a >> 5;
    const int s = k >> 4, r = k & 15;
    const int lane = (int)(a & 31) + 32 * (r >> 3);
    const int j = r & 7;
    return (size_t)b * 32 * d + (size_t)s * 512 + (size_t)lane * 8 + (size_t)j;
}

}  // namespace ebr

using namespace ebr;

extern "C" {

ebr_status ebr_quantize_bf16(const float* in, int64_t n, uint16_t* out) {
    if (n < 0 || (n > 0 && (!in || !out))) { set_error("bad argument"); return EBR_EINVAL; }
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(in[i])) { set_error("non-finite input at %lld", (long long)i); return EBR_EINVAL; }
        out[i] = bf16_rne(in[i]);
    }
    return EBR_OK;
}

ebr_status ebr_quantize_fp8(const float* in, int64_t n, float scale, uint8_t* out) {
    if (n < 0 || (n > 0 && (!in || !out)) || !(scale > 0.0f) || !std::isfinite(scale)) {
        set_error("bad argument");
        return EBR_EINVAL;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(in[i])) { set_error("non-finite input at %lld", (long long)i); return EBR_EINVAL; }
        out[i] = fp8_e4m3_rne(in[i] / scale);
    }
    return EBR_OK;
}

ebr_status ebr_dequantize_fp8(const uint8_t* in, int64_t n, float* out) {
    if (n < 0 || (n > 0 && (!in || !out))) { set_error("bad argument"); return EBR_EINVAL; }
    for (int64_t i = 0; i < n; ++i) out[i] = fp8_e4m3_to_f32(in[i]);
    return EBR_OK;
}

}  // extern "C"
