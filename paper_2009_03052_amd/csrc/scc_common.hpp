// Shared definitions of libscc: exact 128-bit helpers, the per-k lookup tables
// that turn treelet operations into table lookups (the precomputed merge /
// decomposition / colour arrays of Sec. 3.3), device memory and error plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/scc.h"

typedef unsigned __int128 u128;

#define SCC_KMAX 8
#define SCC_MAXSH 128   // r_8 = 115 rooted shapes on 8 nodes

// ---------------------------------------------------------------------------
// Per-k lookup tables, built on the host (treelets.cpp) and copied to the
// device. Colour sets of a vertex v are handled in a (k-1)-colour universe:
// the sets containing c_v (own counts X) and the sets avoiding c_v (neighbour
// sums S) both map to subsets of [k] \ {c_v}, compressed to k-1 bits.
// ---------------------------------------------------------------------------
struct DevLut {
    int k;
    int nkeys;
    int r[SCC_KMAX + 2];        // rooted shapes on h nodes
    int off[SCC_KMAX + 2];      // key offset of level h
    int bk[SCC_KMAX + 2];       // binom(k, h)
    int bk1[SCC_KMAX + 2];      // binom(k-1, h)
    int W[SCC_KMAX + 2];        // own entries per vertex at level h: r_h binom(k-1, h-1)
    int WS[SCC_KMAX + 2];       // neighbour-sum entries at level h: r_h binom(k-1, h)
    int xoff[SCC_KMAX + 2];     // prefix of W over h = 1.. (dense staging offsets)
    int soff[SCC_KMAX + 2];     // prefix of WS over h = 1..
    int num_unr;                // unrooted k-shapes
    uint8_t dec_hp[SCC_KMAX + 1][SCC_MAXSH];   // |T'|
    uint8_t dec_a[SCC_KMAX + 1][SCC_MAXSH];    // rank of T'
    uint8_t dec_b[SCC_KMAX + 1][SCC_MAXSH];    // rank of T''
    uint8_t dec_beta[SCC_KMAX + 1][SCC_MAXSH]; // beta_T
    uint8_t unr_of[SCC_MAXSH];                 // unrooted id of each rooted k-shape
    // Round skipping (Sec. 3.3): the designated rooting of each unrooted k-shape
    // is its smallest rooted rank whose canonical decomposition splits it into
    // two trees of 2..k-2 nodes (-1: the star, which has none; every shape for
    // k < 4); its orbit is the number of nodes of a copy that give that rooting.
    int8_t bal_rank[32];
    uint8_t bal_orbit[32];
    uint8_t designated[SCC_MAXSH];             // 1 for the designated rooted k-shapes
    int star_unr;                              // unrooted id of the k-star
    uint8_t colex_s[128];                      // rank of a (k-1)-bit mask among masks of equal size
    uint8_t mask_s[SCC_KMAX][64];              // [size][rank] -> (k-1)-bit mask
    uint8_t colex_k[256];                      // rank of a k-bit mask among masks of equal size
    uint8_t mask_k[SCC_KMAX + 1][72];          // [size][rank] -> k-bit mask
    // Terms of Eq. (1) in the compressed universe: for a level-h output with
    // colour set D (size h-1, colex rank dc) and |T'| = hp, the i-th split
    // D = D' + D'' (|D'| = hp-1, D' in ascending bitmask order) is
    // (term_x, term_s)[term_base[h][hp] + dc * binom(h-1, hp-1) + i] =
    // (colex rank of D', colex rank of D'').
    uint16_t term_base[SCC_KMAX + 1][SCC_KMAX + 1];
    uint8_t term_x[2200];
    uint8_t term_s[2200];
    // The same, read once per output: output o of level h (o = t binom(k-1, h-1)
    // + dc) has descriptor out[out_off[h] + o] with bits 0-15 the staging offset
    // of its T' block (xoff + rank T' binom(k-1, |T'|-1)), 16-31 that of its T''
    // block, 32-47 its first term, 48-55 its number of splits, 56-62 beta_T and
    // bit 63 set when T is a designated level-k shape; its key at a colour-c
    // vertex is out_key[c][out_off[h] + o]; term_xs[i] = term_x[i] | term_s[i] << 8.
    // (sum over h of W_h is 1376 at k = 8)
    uint32_t out_off[SCC_KMAX + 2];
    uint64_t out[1400];
    uint16_t out_key[SCC_KMAX][1400];
    uint16_t term_xs[2200];
};

// Host-side treelet algebra (treelets.cpp).
struct HostShapes {
    int r[SCC_KMAX + 1];
    uint32_t bits[SCC_KMAX + 1][SCC_MAXSH];   // DFS bitstring, 2(h-1) bits, first edge = MSB
};
const HostShapes &host_shapes();
void build_lut(int k, DevLut *out);
int unrooted_count(int k);
// Unrooted shape id of a tree on k labelled vertices given by adjacency masks.
int tree_unrooted_id(int k, const uint32_t *adjmask);

// ---------------------------------------------------------------------------
// Exact arithmetic helpers (host and device)
// ---------------------------------------------------------------------------
__host__ __device__ inline u128 mk128(uint64_t lo, uint64_t hi) { return ((u128)hi << 64) | lo; }
__host__ __device__ inline uint64_t lo64(u128 x) { return (uint64_t)x; }
__host__ __device__ inline uint64_t hi64(u128 x) { return (uint64_t)(x >> 64); }
__host__ __device__ inline u128 sat_add(u128 a, u128 b)
{
    u128 s = a + b;
    return s < a ? ~(u128)0 : s;
}
__host__ __device__ inline u128 sat_mul(u128 a, u128 b)
{
    if (a == 0 || b == 0) return 0;
    uint64_t ah = hi64(a), bh = hi64(b);
    if (ah && bh) return ~(u128)0;
    // one factor fits in 64 bits
    u128 big = ah ? a : b;
    uint64_t sm = ah ? lo64(b) : lo64(a);
    u128 plo = (u128)lo64(big) * sm;
    u128 phi = (u128)hi64(big) * sm;
    if (hi64(phi)) return ~(u128)0;
    u128 sh = phi << 64;
    return sat_add(plo, sh);
}
// The inverse of an odd d modulo 2^128, by Newton's iteration x <- x (2 - d x)
// (each step doubles the correct low bits; x = d is right to 3 bits).
__host__ __device__ constexpr u128 inv_odd128(uint32_t d)
{
    u128 x = d;
    for (int i = 0; i < 7; i++) x *= (u128)2 - (u128)d * x;
    return x;
}
// x / d for a small d (1..8) that divides x exactly (exact division, Granlund
// and Montgomery, PLDI'94): the factors of two are shifted out, then the odd
// part is a multiplication by its inverse modulo 2^128 (or 2^64). The result
// is meaningless when d does not divide x.
__host__ __device__ inline u128 div_exact_small(u128 x, uint32_t d)
{
    const int s = d & 1u ? 0 : (d & 2u ? 1 : (d & 4u ? 2 : 3));
    const uint32_t o = d >> s;
    x >>= s;
    if (o == 1) return x;
    return x * (o == 3 ? inv_odd128(3) : o == 5 ? inv_odd128(5) : inv_odd128(7));
}
__host__ __device__ inline uint64_t div_exact_small64(uint64_t x, uint32_t d)
{
    const int s = d & 1u ? 0 : (d & 2u ? 1 : (d & 4u ? 2 : 3));
    const uint32_t o = d >> s;
    x >>= s;
    if (o == 1) return x;
    return x * (uint64_t)(o == 3 ? inv_odd128(3) : o == 5 ? inv_odd128(5) : inv_odd128(7));
}
// floor(x / d) for a small divisor d (1..8), by 32-bit long division.
__host__ __device__ inline u128 div_small(u128 x, uint32_t d)
{
    uint64_t h = hi64(x), l = lo64(x);
    uint64_t q3 = (h >> 32) / d, r = (h >> 32) % d;
    uint64_t t = (r << 32) | (h & 0xffffffffu);
    uint64_t q2 = t / d; r = t % d;
    t = (r << 32) | (l >> 32);
    uint64_t q1 = t / d; r = t % d;
    t = (r << 32) | (l & 0xffffffffu);
    uint64_t q0 = t / d;
    return mk128((q1 << 32) | q0, (q3 << 32) | q2);
}
__host__ __device__ inline int bitlen128(u128 x)
{
    uint64_t h = hi64(x), l = lo64(x);
    if (h) return 128 - __builtin_clzll(h);
    if (l) return 64 - __builtin_clzll(l);
    return 0;
}

// (k-1)-bit compressed colour sets: drop / insert the bit of colour c.
__host__ __device__ inline uint32_t compress_out(uint32_t m, int c)
{
    return ((m >> (c + 1)) << c) | (m & ((1u << c) - 1u));
}
__host__ __device__ inline uint32_t expand_in(uint32_t m, int c)
{
    return ((m >> c) << (c + 1)) | (m & ((1u << c) - 1u));
}

// ---------------------------------------------------------------------------
// Errors and device memory
// ---------------------------------------------------------------------------
scc_status set_error(scc_status st, const char *fmt, ...);

#define HIP_TRY(expr)                                                             \
    do {                                                                          \
        hipError_t _e = (expr);                                                   \
        if (_e != hipSuccess)                                                     \
            return set_error(SCC_EDEVICE, "%s failed: %s (%s:%d)", #expr,         \
                             hipGetErrorString(_e), __FILE__, __LINE__);          \
    } while (0)

struct DevMem {
    const scc_allocator *alloc = nullptr;
    hipStream_t stream = nullptr;
    void *get(size_t bytes);
    void put(void *p);
};

// Checks a CSR (sorted, symmetric, simple rows; row_ptr from 0 to nnz) and its
// colours (below k) on the device; SCC_EINVAL on a violation (dp.hip).
scc_status validate_csr(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                        const uint8_t *colors, int k, hipStream_t stream, DevMem &mem);

// Device buffer owned by a table; freed through the same allocator.
struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11). Multipliers and Weyl
// increments as published for the 4x64 variant.
__host__ __device__ inline void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; r++) {
        u128 p0 = (u128)M0 * c[0];
        u128 p1 = (u128)M1 * c[2];
        uint64_t n0 = hi64(p1) ^ c[1] ^ k0;
        uint64_t n2 = hi64(p0) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo64(p1);
        c[2] = n2;
        c[3] = lo64(p0);
        k0 += W0;
        k1 += W1;
    }
}

// Uniform integer in [0, N): Philox key (seed, stream), counter (idx, draw << 32
// | attempt, 0, 0); low 128 output bits masked to bitlen(N-1), rejected if >= N.
__host__ __device__ inline u128 draw_below(u128 N, uint64_t seed, uint64_t stream, uint64_t idx, uint32_t draw)
{
    if (N <= 1) return 0;
    int bits = bitlen128(N - 1);
    u128 mask = bits >= 128 ? ~(u128)0 : (((u128)1 << bits) - 1);
    // each attempt is rejected with probability < 1/2; the cap only guarantees
    // termination and is never reached (probability below 2^-4096)
    for (uint32_t att = 0; att < 4096u; att++) {
        uint64_t c[4] = {idx, ((uint64_t)draw << 32) | att, 0, 0};
        philox4x64_10(c, seed, stream);
        u128 x = mk128(c[0], c[1]) & mask;
        if (x < N) return x;
    }
    return N - 1;
}
