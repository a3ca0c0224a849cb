// Device-side index build (build.hip): argument block and launchers.
#pragma once

#include <cstdint>

#include "internal.h"

namespace ebr {

struct BuildArgs {
    // inputs, device memory
    int64_t n_ads;
    int32_t dim;
    int64_t n_keys;
    const int64_t* key_offsets;   // n_keys + 1
    const uint32_t* post_ids;
    const float* post_w;          // null: no weights (binary L)
    const float* emb;             // n_ads x dim, row-major
    // scratch
    uint32_t* key_chunks;         // n_keys + 1: chunks per list
    uint32_t* key_chunk_off;      // n_keys + 1: their exclusive prefix
    float* key_maxw;              // n_keys: max |w| per list
    uint32_t* chunk_key;          // per chunk: its list
    uint32_t* chunk_words;        // n_chunks + 1: packed words per chunk
    uint32_t* word_off;           // n_chunks + 1: their exclusive prefix
    uint32_t* chunk_info;         // per chunk: b | count << 8
    unsigned long long* flags;    // [0] smallest invalid list, [1] smallest non-finite row (~0: none)
    unsigned long long* stats;    // FP64 bits: max |e|^2, max |e - bf16|^2, max |bf16|^2,
                                  // max |e - fp8|^2, max |fp8|^2 over the ad rows
    int64_t n_chunks;
    // outputs, in the arena
    ChunkHdr* hdr;
    uint32_t* words;
    float* emb_f32;
    uint16_t* emb_bf16;           // null: no BF16 copy
    uint8_t* emb_fp8;             // null: no FP8 copy
    float* fp8_scale;
};

int launch_build_lists(const BuildArgs& a, void* stream);
int launch_build_chunks(const BuildArgs& a, void* stream);  // chunk -> list, then chunk shapes
int launch_build_pack(const BuildArgs& a, void* stream);
int launch_build_rows(const BuildArgs& a, void* stream);
int launch_build_layout(const BuildArgs& a, void* stream);

}  // namespace ebr
