// Posting-list codec (host side).
//
// The paper compresses each inverted list by grouping ids into 256-id blocks
// that share their high 24 bits and storing 8-bit low parts, then padding
// blocks into log2 size groups (Section 3.4, "Block Grouping", "Logarithmic
// Categorization", "Block Compression"; Algorithm 1). This codec keeps the
// goal (fewer bytes per id, load-balanced decode) but is laid out for a
// 64-wide wavefront: each list is cut into chunks of 64 consecutive postings,
// one posting per lane. A chunk stores its first id in a 16-byte header and
// the remaining count - 1 gaps (id_i - id_{i-1} - 1) bit-packed at the
// chunk's own width b, LSB first, so a wave decodes a chunk with one or two
// 32-bit loads per lane plus a wave-wide prefix sum. Chunks hold exact counts:
// nothing is padded, so no padding entry can ever be scattered.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace ebr {

static inline int bit_width(uint32_t v) { return v ? 32 - __builtin_clz(v) : 0; }

static inline void chunk_shape(const uint32_t* ids, int cnt, int* bits, int64_t* words) {
    uint32_t mx = 0;
    for (int i = 1; i < cnt; ++i) mx = std::max(mx, ids[i] - ids[i - 1] - 1u);
    *bits = bit_width(mx);
    *words = ((int64_t)(cnt - 1) * (*bits) + 31) / 32;
}

void codec_measure(const uint32_t* ids, int64_t n, int64_t* chunks, int64_t* words) {
    int64_t c = 0, w = 0;
    for (int64_t s = 0; s < n; s += kChunk) {
        int cnt = (int)std::min<int64_t>(kChunk, n - s);
        int b;
        int64_t nw;
        chunk_shape(ids + s, cnt, &b, &nw);
        ++c;
        w += nw;
    }
    *chunks = c;
    *words = w;
}

void codec_encode(const uint32_t* ids, int64_t n, ChunkHdr* hdr, uint32_t* words,
                  uint32_t word_base, uint32_t post_base) {
    int64_t wcur = 0;
    for (int64_t s = 0, c = 0; s < n; s += kChunk, ++c) {
        int cnt = (int)std::min<int64_t>(kChunk, n - s);
        int b;
        int64_t nw;
        chunk_shape(ids + s, cnt, &b, &nw);
        hdr[c].first_id = ids[s];
        hdr[c].info = (uint32_t)b | ((uint32_t)cnt << 8);
        hdr[c].word_off = word_base + (uint32_t)wcur;
        hdr[c].post_off = post_base + (uint32_t)s;
        uint32_t* w = words + wcur;
        std::memset(w, 0, (size_t)nw * 4);
        for (int i = 1; i < cnt; ++i) {
            uint64_t gap = (uint64_t)(ids[s + i] - ids[s + i - 1] - 1u);
            uint64_t bitpos = (uint64_t)(i - 1) * (uint64_t)b;
            uint64_t v = gap << (bitpos & 31);
            w[bitpos >> 5] |= (uint32_t)v;
            if ((v >> 32) != 0) w[(bitpos >> 5) + 1] |= (uint32_t)(v >> 32);
        }
        wcur += nw;
    }
}

bool codec_decode(const ChunkHdr* hdr, int64_t n_chunks, const uint32_t* words,
                  int64_t n_words, int64_t n, uint32_t* ids) {
    int64_t pos = 0;
    for (int64_t c = 0; c < n_chunks; ++c) {
        int b = hdr_bits(hdr[c].info), cnt = hdr_count(hdr[c].info);
        if (b > 32 || cnt < 1 || cnt > kChunk || pos + cnt > n) return false;
        if (hdr[c].post_off != (uint32_t)pos) return false;
        int64_t need = ((int64_t)(cnt - 1) * b + 31) / 32;
        if ((int64_t)hdr[c].word_off + need > n_words) return false;
        const uint32_t* w = words + hdr[c].word_off;
        uint64_t cur = hdr[c].first_id;
        ids[pos] = (uint32_t)cur;
        for (int i = 1; i < cnt; ++i) {
            uint64_t bitpos = (uint64_t)(i - 1) * (uint64_t)b;
            uint64_t lo = w[bitpos >> 5];
            uint64_t hi = ((bitpos >> 5) + 1 < (uint64_t)need) ? w[(bitpos >> 5) + 1] : 0;
            uint64_t v = ((hi << 32) | lo) >> (bitpos & 31);
            uint64_t gap = (b == 32) ? (v & 0xffffffffull) : (v & ((1ull << b) - 1));
            cur += gap + 1;
            if (cur > 0xffffffffull) return false;
            ids[pos + i] = (uint32_t)cur;
        }
        pos += cnt;
    }
    return pos == n;
}

}  // namespace ebr
