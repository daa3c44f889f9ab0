// Device-side helpers shared by the libscc kernels (wave64, gfx950).
#pragma once

#include "scc_common.hpp"

#define WAVE 64

// ---------------------------------------------------------------------------
// Table views passed to kernels
// ---------------------------------------------------------------------------
// One stored level h >= 2. The locator of v packs the record's word offset in
// the pool (40 bits), its length (12 bits) and a 128-bit flag (1 bit). The
// record (len entries, sorted by key) is: the vertex's level sum N (2 words),
// ceil(len/4) words of uint16 keys, len words of low count bits and, for a
// 128-bit vertex, len words of high bits. A vertex without entries has
// locator 0 and no record.
struct LevelView {
    const uint64_t *pool;
    const uint64_t *loc;       // [n] record locators
    const uint64_t *bm;        // presence bitmaps, BW words per vertex
    int BW;
    int vlc;                   // records in the variable-length layout (below)
};

#define LOC_OFF(l) ((l) & 0xffffffffffull)
#define LOC_LEN(l) ((uint32_t)(((l) >> 40) & 0xfffu))
#define LOC_WIDE(l) ((uint32_t)(((l) >> 52) & 1u))
#define REC_HDR 2u

// build-time record summary: len | wide << 31
#define META_LEN(m) ((m) & 0x7fffffffu)
#define META_WIDE(m) ((m) >> 31)

__host__ __device__ inline uint32_t key_words(uint32_t len) { return (len + 3u) >> 2; }
__host__ __device__ inline uint64_t make_loc(uint64_t off, uint32_t len, uint32_t wide)
{
    return len ? (off | ((uint64_t)len << 40) | ((uint64_t)wide << 52)) : 0ull;
}

// Variable-length records (Sec. 3.3, "Variable-length counts"): after the
// level sum N, one u16 per entry holding the key (11 bits) and the count's
// length in bytes (5 bits), ceil(len/4) words; then the byte offset of every
// 32nd entry's count (u16 each, ceil(ceil(len/32)/4) words); then the counts,
// little-endian, byte after byte. An entry's offset is its checkpoint plus
// the lengths of the entries between, summed four headers per word.
constexpr uint32_t VLC_CK = 32;
__host__ __device__ inline uint32_t vlc_ck_words(uint32_t len) { return ((len + VLC_CK - 1) / VLC_CK + 3) / 4; }
__device__ inline uint32_t vlc_len4(uint64_t w)
{
    return (uint32_t)((((w >> 11) & 0x001F001F001F001Full) * 0x0001000100010001ull) >> 48);
}
__device__ inline uint32_t vlc_bytes(u128 c)
{
    const int b = bitlen128(c);
    return b ? (uint32_t)(b + 7) / 8 : 1u;
}

struct Rec {
    const uint64_t *p;   // record start (the header)
    uint32_t len, kw;
    bool wide;
    bool vlc;
    __device__ uint32_t key(uint32_t e) const
    {
        const uint32_t h = ((const uint16_t *)(p + REC_HDR))[e];
        return vlc ? (h & 0x7ffu) : h;
    }
    __device__ u128 vcnt(uint32_t e) const
    {
        const uint16_t *hd = (const uint16_t *)(p + REC_HDR);
        const uint32_t ckw = vlc_ck_words(len);
        uint32_t off = ((const uint16_t *)(p + REC_HDR + kw))[e / VLC_CK];
        const uint64_t *hw = p + REC_HDR + (e & ~(VLC_CK - 1)) / 4;
        const uint32_t full = (e % VLC_CK) / 4, rem = e % 4;
        for (uint32_t i = 0; i < full; i++) off += vlc_len4(hw[i]);
        if (rem) off += vlc_len4(hw[full] & ((1ull << (16 * rem)) - 1ull));
        const uint32_t l = hd[e] >> 11;
        const uint64_t *cw = p + REC_HDR + kw + ckw + off / 8;
        const uint32_t sh = (off % 8) * 8, end = off % 8 + l;
        const uint64_t w0 = cw[0], w1 = end > 8 ? cw[1] : 0, w2 = end > 16 ? cw[2] : 0;
        uint64_t lo = sh ? (w0 >> sh) | (w1 << (64 - sh)) : w0;
        uint64_t hi = sh ? (w1 >> sh) | (w2 << (64 - sh)) : w1;
        if (l < 8) { lo &= (1ull << (8 * l)) - 1ull; hi = 0; }
        else if (l == 8) hi = 0;
        else if (l < 16) hi &= (1ull << (8 * (l - 8))) - 1ull;
        return mk128(lo, hi);
    }
    __device__ u128 cnt(uint32_t e) const
    {
        if (vlc) return vcnt(e);
        return mk128(p[REC_HDR + kw + e], wide ? p[REC_HDR + kw + len + e] : 0);
    }
    __device__ uint64_t lo(uint32_t e) const { return lo64(cnt(e)); }
    __device__ uint64_t hi(uint32_t e) const { return hi64(cnt(e)); }
    __device__ u128 N() const { return len ? mk128(p[0], p[1]) : (u128)0; }
};

__device__ inline Rec rec_of(const LevelView &L, int64_t v)
{
    const uint64_t l = L.loc[v];
    Rec r;
    r.len = LOC_LEN(l);
    r.wide = LOC_WIDE(l) != 0;
    r.vlc = L.vlc != 0;
    r.kw = key_words(r.len);
    r.p = L.pool + LOC_OFF(l);
    return r;
}

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

// Wave scans on DPP lane moves (no LDS round trips), all 64 lanes active:
// row_shr 1, 2, 4, 8 scan each row of 16 lanes; row_bcast 15 then adds a row's
// last lane to the next row (rows 1 and 3), row_bcast 31 adds lane 31 to rows 2
// and 3. Lanes a move does not reach, or whose source is outside the row,
// receive 0.
enum { DPP_SHR1 = 0x111, DPP_SHR2 = 0x112, DPP_SHR4 = 0x114, DPP_SHR8 = 0x118, DPP_BC15 = 0x142, DPP_BC31 = 0x143 };

template <int CTRL, int ROWS>
__device__ inline uint32_t dpp32(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xf, true);
}
template <int CTRL, int ROWS>
__device__ inline uint64_t dpp64(uint64_t x)
{
    return ((uint64_t)dpp32<CTRL, ROWS>((uint32_t)(x >> 32)) << 32) | dpp32<CTRL, ROWS>((uint32_t)x);
}
template <int CTRL, int ROWS>
__device__ inline u128 dpp128(u128 x)
{
    return mk128(dpp64<CTRL, ROWS>(lo64(x)), dpp64<CTRL, ROWS>(hi64(x)));
}

__device__ inline u128 wave_incl_scan128(u128 x)
{
    x += dpp128<DPP_SHR1, 0xf>(x);
    x += dpp128<DPP_SHR2, 0xf>(x);
    x += dpp128<DPP_SHR4, 0xf>(x);
    x += dpp128<DPP_SHR8, 0xf>(x);
    x += dpp128<DPP_BC15, 0xa>(x);
    x += dpp128<DPP_BC31, 0xc>(x);
    return x;
}

// inclusive scan that saturates at 2^128 - 1 instead of wrapping
__device__ inline u128 wave_incl_satscan128(u128 x)
{
    x = sat_add(x, dpp128<DPP_SHR1, 0xf>(x));
    x = sat_add(x, dpp128<DPP_SHR2, 0xf>(x));
    x = sat_add(x, dpp128<DPP_SHR4, 0xf>(x));
    x = sat_add(x, dpp128<DPP_SHR8, 0xf>(x));
    x = sat_add(x, dpp128<DPP_BC15, 0xa>(x));
    x = sat_add(x, dpp128<DPP_BC31, 0xc>(x));
    return x;
}

__device__ inline uint32_t wave_incl_scan32(uint32_t x)
{
    x += dpp32<DPP_SHR1, 0xf>(x);
    x += dpp32<DPP_SHR2, 0xf>(x);
    x += dpp32<DPP_SHR4, 0xf>(x);
    x += dpp32<DPP_SHR8, 0xf>(x);
    x += dpp32<DPP_BC15, 0xa>(x);
    x += dpp32<DPP_BC31, 0xc>(x);
    return x;
}

__device__ inline uint64_t wave_incl_scan64(uint64_t x)
{
    x += dpp64<DPP_SHR1, 0xf>(x);
    x += dpp64<DPP_SHR2, 0xf>(x);
    x += dpp64<DPP_SHR4, 0xf>(x);
    x += dpp64<DPP_SHR8, 0xf>(x);
    x += dpp64<DPP_BC15, 0xa>(x);
    x += dpp64<DPP_BC31, 0xc>(x);
    return x;
}

__device__ inline uint32_t wave_incl_max32(uint32_t x)
{
    x = max(x, dpp32<DPP_SHR1, 0xf>(x));
    x = max(x, dpp32<DPP_SHR2, 0xf>(x));
    x = max(x, dpp32<DPP_SHR4, 0xf>(x));
    x = max(x, dpp32<DPP_SHR8, 0xf>(x));
    x = max(x, dpp32<DPP_BC15, 0xa>(x));
    x = max(x, dpp32<DPP_BC31, 0xc>(x));
    return x;
}

// value of lane 63, uniform
__device__ inline uint64_t last_lane64(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, WAVE - 1);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), WAVE - 1);
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline u128 last_lane128(u128 x) { return mk128(last_lane64(lo64(x)), last_lane64(hi64(x))); }
// value of the first active lane, in every lane (scalar)
__device__ inline uint64_t readfirst64(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}
// value of lane src (uniform src), in every lane
__device__ inline uint64_t readlane64(uint64_t x, int src)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// totals over the wave, in every lane
__device__ inline u128 wave_sum128(u128 x) { return last_lane128(wave_incl_scan128(x)); }
__device__ inline u128 wave_satsum128(u128 x) { return last_lane128(wave_incl_satscan128(x)); }
__device__ inline uint64_t wave_sum64(uint64_t x) { return last_lane64(wave_incl_scan64(x)); }

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
    return rec_of(L, v).cnt(pos);
}

// Count of a key in a stored record by binary search (0 if absent).
__device__ inline u128 record_lookup(const LevelView &L, int64_t v, uint32_t key)
{
    const Rec r = rec_of(L, v);
    uint32_t lo = 0, hi = r.len;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        const uint32_t kk = r.key(mid);
        if (kk == key) return r.cnt(mid);
        if (kk < key) lo = mid + 1; else hi = mid;
    }
    return 0;
}
