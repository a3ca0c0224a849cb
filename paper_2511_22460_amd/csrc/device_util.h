// Device helpers shared by the gfx950 kernels of libebr (wave-level scans, orderable score
// keys, BF16 rounding).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"
#include "kernels.h"

namespace ebr {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------------ small helpers

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = lane_id();
    #pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Orderable key of an FP32 score: larger score <=> larger key; -0.0 maps like +0.0.
__device__ __forceinline__ uint32_t score_key(float s) {
    uint32_t u = __float_as_uint(s + 0.0f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_score(uint32_t k) {
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

// Block-wide exclusive scan for blockDim.x == NT (multiple of 64). sbuf holds NT/64 + 1 words.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sbuf, uint32_t* total) {
    constexpr int NW = NT / 64;
    const int lane = lane_id(), wave = (int)(threadIdx.x >> 6);
    uint32_t incl = wave_incl_scan(v);
    if (lane == 63) sbuf[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < NW; ++w) {
            uint32_t t = sbuf[w];
            sbuf[w] = run;
            run += t;
        }
        sbuf[NW] = run;
    }
    __syncthreads();
    uint32_t r = incl - v + sbuf[wave];
    *total = sbuf[NW];
    __syncthreads();
    return r;
}

// Inclusive prefix maximum over the 64 lanes (values >= -1) with DPP moves: shifts by 1, 2, 4
// and 8 within each row of 16 lanes, then row 15 / row 31 broadcasts into the later rows.
__device__ __forceinline__ int wave_incl_max(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return v;
}

// Inclusive prefix sum over the 64 lanes, same DPP pattern.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
    return v;
}

// Whether a query's 32-bit cross term is precise enough for its result: the rounding bound
// werr (half a quantum per feature) against the returned scores g0 >= ... >= gk must stay
// within kWideTau of the smallest returned magnitude (gk for positive scores, |g0| for
// negative ones, zero when the scores change sign).
__device__ __forceinline__ bool wide_precise(float werr, float g0, float gk) {
    const float mn = gk > 0.0f ? gk : (g0 < 0.0f ? -g0 : 0.0f);
    return werr <= kWideTau * mn;
}

// FP32 -> BF16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// The kth largest (k >= 1) of the n distinct keys s[0, n): an MSB-first radix select, one
// byte per pass (LDS histogram of the keys that share the bytes fixed so far).
__device__ __forceinline__ unsigned long long kth_largest(const unsigned long long* s, int n, int kth, uint32_t* hist,
                                          unsigned long long* pref, int* rank_out) {
    const int tid = (int)threadIdx.x;
    unsigned long long prefix = 0ull, mask = 0ull;
    int rank = kth;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = tid; b < 256; b += (int)blockDim.x) hist[b] = 0u;
        __syncthreads();
        for (int i = tid; i < n; i += (int)blockDim.x) {
            const unsigned long long key = s[i];
            if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (tid < 64) {
            // lane l: bins 255 - 4 l .. 252 - 4 l, counted from the top
            uint32_t v[4], sum = 0u;
            #pragma unroll
            for (int t = 0; t < 4; ++t) {
                v[t] = hist[255 - (4 * tid + t)];
                sum += v[t];
            }
            const uint32_t incl = wave_incl_sum(sum);
            uint32_t acc = incl - sum;
            if (acc < (uint32_t)rank && (uint32_t)rank <= incl) {
                #pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (acc < (uint32_t)rank && (uint32_t)rank <= acc + v[t]) {
                        *pref = prefix | ((unsigned long long)(255 - (4 * tid + t)) << shift);
                        *rank_out = rank - (int)acc;
                    }
                    acc += v[t];
                }
            }
        }
        __syncthreads();
        prefix = *pref;
        rank = *rank_out;
        mask |= 255ull << shift;
        __syncthreads();
    }
    return prefix;
}

}  // namespace ebr
