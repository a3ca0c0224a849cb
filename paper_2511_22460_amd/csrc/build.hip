// Device-side index build for online refresh: the same arena bytes as the host build
// (ebr_build_index), computed on the GPU from posting lists and embeddings that are already in
// device memory. The paper rebuilds its GPU inverted list whenever the feature-to-ad matrix
// changes (Section 3.4) and builds it with parallel grouping and partitioning (Algorithm 1);
// here the lists are cut into the same 64-posting chunks as the host codec (codec.cpp):
//   k_bld_lists  - per list: ids strictly increasing and < N, weights finite, max |w|, chunks
//   scan         - chunk offsets per list
//   k_bld_chunks - per chunk: its list
//   k_bld_shape  - per chunk: gap bit width b and packed words
//   scan         - word offsets per chunk
//   k_bld_pack   - per chunk: header and packed gap words
//   k_bld_rows   - per ad row: finite check, row norms and quantisation errors (FP64), FP8 scale
//   k_bld_layout - the FP32 copy (row-major, padded to whole tiles), BF16 / FP8 in the 32x32x16
//                  operand layout
#include <hip/hip_runtime.h>

#include <cmath>

#include "build.h"
#include "device_util.h"

namespace ebr {

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    #pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

__device__ __forceinline__ float wave_max_f32(float v) {
    #pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// BF16 round to nearest even (the bits of the FP32 pattern, as quant.cpp)
__device__ __forceinline__ uint16_t bld_bf16(float x) {
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// OCP e4m3fn code of a finite x, round to nearest even, saturating to +-448 (as quant.cpp)
__device__ __forceinline__ uint8_t bld_fp8(float x) {
    const uint8_t sign = signbit(x) ? 0x80 : 0x00;
    const double a = fabs((double)x);
    if (a >= 448.0) return sign | 0x7e;
    if (a < 0x1p-6) return sign | (uint8_t)rint(ldexp(a, 9));  // subnormals: multiples of 2^-9
    int e;
    const double f = frexp(a, &e);  // a = f 2^e, f in [0.5, 1)
    int ex = e - 1;
    double m = rint((2.0 * f - 1.0) * 8.0);
    if (m >= 8.0) { m = 0.0; ++ex; }
    if (ex > 8 || (ex == 8 && m > 6.0)) return sign | 0x7e;
    return sign | (uint8_t)(((ex + 7) << 3) | (int)m);
}

__device__ __forceinline__ double bld_fp8_value(uint8_t c) {
    const int s = c >> 7, e = (c >> 3) & 15, m = c & 7;
    const double v = e == 0 ? ldexp((double)m, -9) : ldexp(1.0 + m / 8.0, e - 7);
    return s ? -v : v;
}

__device__ __forceinline__ void max_u64(unsigned long long* p, double v) {
    atomicMax(p, (unsigned long long)__double_as_longlong(v));  // v >= 0: bits order as values
}

// One wavefront per list (grid-stride): validity, max |w| (1 for a list without weights),
// chunk count.
__global__ __launch_bounds__(256) void k_bld_lists(BuildArgs a) {
    const int lane = lane_id();
    const int64_t w0 = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6), nw = (int64_t)gridDim.x * 4;
    for (int64_t k = w0; k < a.n_keys; k += nw) {
        const int64_t s = a.key_offsets[k], t = a.key_offsets[k + 1];
        bool bad = false;
        float mx = 0.0f;
        for (int64_t i = s + lane; i < t; i += 64) {
            const uint32_t id = a.post_ids[i];
            if ((int64_t)id >= a.n_ads || (i > s && a.post_ids[i - 1] >= id)) bad = true;
            if (a.post_w) {
                const float x = a.post_w[i];
                if (!isfinite(x)) bad = true;
                mx = fmaxf(mx, fabsf(x));
            }
        }
        bad = __ballot(bad) != 0ull;
        mx = wave_max_f32(mx);
        if (lane == 0) {
            a.key_chunks[k] = (uint32_t)((t - s + 63) / 64);
            a.key_maxw[k] = a.post_w ? mx : (t > s ? 1.0f : 0.0f);
            if (bad) atomicMin(&a.flags[0], (unsigned long long)k);
        }
    }
}

// One wavefront per list: chunk c of list k is chunk key_chunk_off[k] + c of the index.
__global__ __launch_bounds__(256) void k_bld_chunks(BuildArgs a) {
    const int lane = lane_id();
    const int64_t w0 = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6), nw = (int64_t)gridDim.x * 4;
    for (int64_t k = w0; k < a.n_keys; k += nw) {
        const uint32_t c0 = a.key_chunk_off[k], n = a.key_chunk_off[k + 1] - c0;
        for (uint32_t c = (uint32_t)lane; c < n; c += 64u) a.chunk_key[c0 + c] = (uint32_t)k;
    }
}

// This lane's posting of chunk c: its id and gap (id - previous id - 1; lane 0 and lanes past
// the chunk: 0), the chunk's first posting and count.
struct ChunkLane {
    uint32_t id, gap;
    int64_t i0;
    int cnt;
};

__device__ __forceinline__ ChunkLane chunk_lane(const BuildArgs& a, int64_t c) {
    const int lane = lane_id();
    const uint32_t k = a.chunk_key[c];
    ChunkLane r;
    r.i0 = a.key_offsets[k] + 64 * (c - (int64_t)a.key_chunk_off[k]);
    r.cnt = (int)min((int64_t)64, a.key_offsets[k + 1] - r.i0);
    r.id = lane < r.cnt ? a.post_ids[r.i0 + lane] : 0u;
    const uint32_t prev = (uint32_t)__shfl_up((int)r.id, 1, 64);
    r.gap = (lane >= 1 && lane < r.cnt) ? r.id - prev - 1u : 0u;
    return r;
}

// One wavefront per chunk: gap width b (the largest gap's bit count) and packed words.
__global__ __launch_bounds__(256) void k_bld_shape(BuildArgs a) {
    const int64_t w0 = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6), nw = (int64_t)gridDim.x * 4;
    for (int64_t c = w0; c < a.n_chunks; c += nw) {
        const ChunkLane r = chunk_lane(a, c);
        const uint32_t mx = wave_max_u32(r.gap);
        const int b = mx ? 32 - __builtin_clz(mx) : 0;
        if (lane_id() == 0) {
            a.chunk_words[c] = (uint32_t)(((int64_t)(r.cnt - 1) * b + 31) / 32);
            a.chunk_info[c] = (uint32_t)b | ((uint32_t)r.cnt << 8);
        }
    }
}

// One wavefront per chunk: its header and gap words (gap i of the chunk at bit (i - 1) b of
// the chunk's words, LSB first); word w is assembled by lane w from the gaps it overlaps.
__global__ __launch_bounds__(256) void k_bld_pack(BuildArgs a) {
    __shared__ uint32_t s_gap[4][64];
    const int lane = lane_id(), wv = (int)(threadIdx.x >> 6);
    const int64_t w0 = (int64_t)blockIdx.x * 4 + wv, nw = (int64_t)gridDim.x * 4;
    for (int64_t c = w0; c < a.n_chunks; c += nw) {
        const ChunkLane r = chunk_lane(a, c);
        const uint32_t info = a.chunk_info[c];
        const int b = (int)(info & 63u);
        const uint32_t woff = a.word_off[c], nwords = a.word_off[c + 1] - woff;
        if (lane == 0) {
            ChunkHdr h;
            h.first_id = r.id;
            h.info = info;
            h.word_off = woff;
            h.post_off = (uint32_t)r.i0;
            a.hdr[c] = h;
        }
        s_gap[wv][lane] = r.gap;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        if ((uint32_t)lane < nwords) {
            const int lo = 32 * lane, hi = lo + 31;  // this word's bits
            uint32_t word = 0u;
            for (int g = lo / b; g <= min(r.cnt - 2, hi / b); ++g) {  // gap g + 1 at bit g b
                const uint32_t v = s_gap[wv][g + 1];
                const int rel = g * b - lo;
                word |= rel >= 0 ? (v << rel) : (v >> (-rel));
            }
            a.words[woff + (uint32_t)lane] = word;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// One thread per ad row slot of the copies (rows >= n_ads: the padding of the last block).
__global__ __launch_bounds__(256) void k_bld_rows(BuildArgs a, int64_t n_rows) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    if (r >= a.n_ads) {
        if (a.fp8_scale) a.fp8_scale[r] = 1.0f;
        return;
    }
    const float* row = a.emb + r * a.dim;
    double n2 = 0.0, mx = 0.0;
    bool bad = false;
    for (int k = 0; k < a.dim; ++k) {
        const float x = row[k];
        if (!isfinite(x)) bad = true;
        n2 += (double)x * x;
        mx = fmax(mx, fabs((double)x));
    }
    if (bad) {
        atomicMin(&a.flags[1], (unsigned long long)r);
        return;
    }
    max_u64(&a.stats[0], n2);
    if (a.emb_bf16) {
        double er = 0.0, nr = 0.0;
        for (int k = 0; k < a.dim; ++k) {
            const double q = (double)__uint_as_float((uint32_t)bld_bf16(row[k]) << 16);
            er += (q - row[k]) * (q - row[k]);
            nr += q * q;
        }
        max_u64(&a.stats[1], er);
        max_u64(&a.stats[2], nr);
    }
    if (a.emb_fp8) {
        const float sc = mx > 0.0 ? (float)(mx / 448.0) : 1.0f;
        a.fp8_scale[r] = sc;
        double er = 0.0, nr = 0.0;
        for (int k = 0; k < a.dim; ++k) {
            // x / sc rounded once to FP32: the FP64 quotient of two FP32 values rounds to the
            // same FP32 value as an FP32 division (53 >= 2 * 24 + 2 bits)
            const uint8_t c8 = bld_fp8((float)((double)row[k] / (double)sc));
            const double q = (double)sc * (double)(float)bld_fp8_value(c8);
            er += (q - row[k]) * (q - row[k]);
            nr += q * q;
        }
        max_u64(&a.stats[3], er);
        max_u64(&a.stats[4], nr);
    }
}

// One thread per element of a 32-ad block of the copies.
__global__ __launch_bounds__(256) void k_bld_layout(BuildArgs a, int64_t n_elem) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_elem) return;
    const int d = a.dim;
    const int64_t blk = idx / (32 * d);
    const int r = (int)(idx % (32 * d));
    {
        // FP32: the rows, row-major, zero rows past the inventory
        const int64_t row = 32 * blk + r / d;
        a.emb_f32[idx] = row < a.n_ads ? a.emb[idx] : 0.0f;
    }
    if (a.emb_bf16 || a.emb_fp8) {
        // 16-dim step s, lane l, value j holds e[32 blk + (l & 31)][16 s + 8 (l >> 5) + j]
        const int s = r / 512, l = (r / 8) % 64, j = r % 8;
        const int64_t row = 32 * blk + (l & 31);
        const int col = 16 * s + 8 * (l >> 5) + j;
        const bool in = row < a.n_ads;
        const float x = in ? a.emb[row * d + col] : 0.0f;
        if (a.emb_bf16) a.emb_bf16[idx] = in ? bld_bf16(x) : (uint16_t)0;
        if (a.emb_fp8) a.emb_fp8[idx] = in ? bld_fp8((float)((double)x / (double)a.fp8_scale[row])) : (uint8_t)0;
    }
}

static int bld_last(hipError_t e) { return e == hipSuccess ? (int)hipGetLastError() : (int)e; }

static unsigned grid_waves(int64_t n) {
    const int64_t blocks = (n + 3) / 4;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, 65536));
}

int launch_build_lists(const BuildArgs& a, void* stream) {
    if (a.n_keys <= 0) return 0;
    hipLaunchKernelGGL(k_bld_lists, dim3(grid_waves(a.n_keys)), dim3(256), 0, (hipStream_t)stream, a);
    return bld_last(hipSuccess);
}

int launch_build_chunks(const BuildArgs& a, void* stream) {
    if (a.n_keys <= 0 || a.n_chunks <= 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_bld_chunks, dim3(grid_waves(a.n_keys)), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_bld_shape, dim3(grid_waves(a.n_chunks)), dim3(256), 0, st, a);
    return bld_last(hipSuccess);
}

int launch_build_pack(const BuildArgs& a, void* stream) {
    if (a.n_chunks <= 0) return 0;
    hipLaunchKernelGGL(k_bld_pack, dim3(grid_waves(a.n_chunks)), dim3(256), 0, (hipStream_t)stream, a);
    return bld_last(hipSuccess);
}

int launch_build_rows(const BuildArgs& a, void* stream) {
    const int64_t n_rows = (a.n_ads + 31) / 32 * 32;
    hipLaunchKernelGGL(k_bld_rows, dim3((unsigned)((n_rows + 255) / 256)), dim3(256), 0, (hipStream_t)stream, a, n_rows);
    return bld_last(hipSuccess);
}

int launch_build_layout(const BuildArgs& a, void* stream) {
    const int64_t n_elem = (a.n_ads + 31) / 32 * 32 * a.dim;
    hipLaunchKernelGGL(k_bld_layout, dim3((unsigned)((n_elem + 255) / 256)), dim3(256), 0, (hipStream_t)stream, a, n_elem);
    return bld_last(hipSuccess);
}

}  // namespace ebr
