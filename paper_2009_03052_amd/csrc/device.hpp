// Device-side helpers shared by the libscc kernels (wave64, gfx950).
#pragma once

#include "scc_common.hpp"

#define WAVE 64

// ---------------------------------------------------------------------------
// Table views passed to kernels
// ---------------------------------------------------------------------------
// One stored level h >= 2. Record of v (len entries, sorted by key) starts at
// word off[v] of pool: ceil(len/4) words of uint16 keys, then len words of low
// count bits, then, if the vertex is wide, len words of high bits.
struct LevelView {
    const uint64_t *pool;
    const uint64_t *off;
    const uint32_t *meta;      // len | wide << 31
    const u128 *N;             // sum of the vertex's counts at this level
    const uint64_t *bm;        // presence bitmaps, BW words per vertex
    int BW;
};

#define META_LEN(m) ((m) & 0x7fffffffu)
#define META_WIDE(m) ((m) >> 31)

__device__ inline uint32_t key_words(uint32_t len) { return (len + 3u) >> 2; }

struct GraphView {
    int64_t n;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    const uint8_t *colors;
};

// ---------------------------------------------------------------------------
// Wave primitives
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }

__device__ inline uint64_t shfl64(uint64_t x, int src)
{
    return (uint64_t)__shfl((unsigned long long)x, src, WAVE);
}
__device__ inline u128 shfl128(u128 x, int src) { return mk128(shfl64(lo64(x), src), shfl64(hi64(x), src)); }

__device__ inline u128 wave_incl_scan128(u128 x)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        uint64_t l = (uint64_t)__shfl_up((unsigned long long)lo64(x), d, WAVE);
        uint64_t h = (uint64_t)__shfl_up((unsigned long long)hi64(x), d, WAVE);
        if (lane >= d) x += mk128(l, h);
    }
    return x;
}

__device__ inline uint32_t wave_incl_scan32(uint32_t x)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        uint32_t y = __shfl_up(x, d, WAVE);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ inline u128 wave_sum128(u128 x)
{
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1)
        x += mk128(shfl64(lo64(x), lane_id() ^ d), shfl64(hi64(x), lane_id() ^ d));
    return x;
}

__device__ inline u128 wave_satsum128(u128 x)
{
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1)
        x = sat_add(x, mk128(shfl64(lo64(x), lane_id() ^ d), shfl64(hi64(x), lane_id() ^ d)));
    return x;
}

__device__ inline uint64_t wave_sum64(uint64_t x)
{
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1) x += shfl64(x, lane_id() ^ d);
    return x;
}

__device__ inline uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// Count of the entry with dense level position li (>= 0) at v, via the presence
// bitmap: its rank among v's present entries is its position in the record.
__device__ inline u128 record_at(const LevelView &L, int64_t v, int li)
{
    const uint64_t *bw = L.bm + (size_t)v * L.BW;
    const int w = li >> 6;
    const uint64_t word = bw[w];
    if (!((word >> (li & 63)) & 1ull)) return 0;
    uint32_t pos = (uint32_t)__popcll(word & ((1ull << (li & 63)) - 1ull));
    for (int q = 0; q < w; q++) pos += (uint32_t)__popcll(bw[q]);
    const uint32_t m = L.meta[v], len = META_LEN(m);
    const uint64_t *rec = L.pool + L.off[v];
    const uint32_t kw = key_words(len);
    return mk128(rec[kw + pos], META_WIDE(m) ? rec[kw + len + pos] : 0);
}

// Count of a key in a stored record by binary search (0 if absent).
__device__ inline u128 record_lookup(const LevelView &L, int64_t v, uint32_t key)
{
    uint32_t m = L.meta[v];
    uint32_t len = META_LEN(m);
    if (len == 0) return 0;
    const uint64_t *rec = L.pool + L.off[v];
    const uint16_t *keys = (const uint16_t *)rec;
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        uint32_t kk = keys[mid];
        if (kk == key) {
            uint32_t kw = key_words(len);
            uint64_t cl = rec[kw + mid];
            uint64_t ch = META_WIDE(m) ? rec[kw + len + mid] : 0;
            return mk128(cl, ch);
        }
        if (kk < key) lo = mid + 1; else hi = mid;
    }
    return 0;
}
