// Build-up phase for k up to 16 (Sec. 3.2): rooted treelets as DFS
// bitstrings, the count table of every vertex as a sorted list of (coloured
// treelet, count) pairs holding only the non-zero counts, and Eq. (1)
// evaluated on those lists.
//
// Keys. A rooted treelet T on h nodes is its DFS bitstring s_T of 2(h-1) bits
// ('1' away from the root, '0' back; the root's child words "1 s 0" in
// descending lexicographic order; first edge at the most significant bit). A
// coloured treelet (T, C) is exported as key = s_T << 16 | C, C the k-bit
// colour mask (46 bits at most).
//
// Levels. X_h holds at each vertex the non-zero c(T_C, v), |T| = h, sorted by
// key. S_j holds at each vertex v the neighbour sums sum_{u ~ v} c(T_C, u)
// over colour sets C that avoid c_v, sorted colour-major (C, then s_T), so that
// the combine finds every sum of one colour set by binary search.
//
// Eq. (1) with T'' the largest root child: every T on h nodes arises from
// exactly one pair (T', T'') where T = w(T'') s_T' (the word w = "1 s_T'' 0"
// put in front of T''s string) and w is not smaller than the first root
// child word of T'; beta_T is then the number of T's root child words equal to
// its first one.
//
// Work is formed as terms and aggregated by sorting. Each level (X_h, and
// the sums S_h built from it) first counts its terms per vertex -- neighbour
// entries for S_h, non-zero products of Eq. (1) for X_h -- then, a chunk of
// vertices at a time, writes each term as one 64-bit word (vertex in the
// chunk above the sort key) with its count, sorts the words (least
// significant digit radix sort, 8-bit digits, stable), adds the counts of
// equal words and, for X_h, divides each sum by beta_T. Counts are exact
// unsigned integers of 128 bits, or of 256 bits when a build needs them (every
// kernel that carries counts is instantiated for both widths); a product or sum
// that needs more bits than the build's width ends it with SCC_EOVERFLOW.
#include <algorithm>
#include <vector>

#include "device.hpp"

namespace {

constexpr int K16 = 16;
constexpr int WPB = 4;                      // waves per block
constexpr int BLOCK = WPB * WAVE;           // 256 threads
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;   // elements per scan block
constexpr int RADIX_BITS = 8;                   // digit width of the radix sort
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int SORT_ITEMS = 16;
constexpr int SORT_TILE = BLOCK * SORT_ITEMS;   // elements per sort block
constexpr int64_t DEFAULT_CHUNK_TERMS = (int64_t)1 << 26;
constexpr int64_t MAX_CHUNK_TERMS = ((int64_t)1 << 31) - 1;   // sort permutations are uint32

enum { E16_OVERFLOW = 1, E16_BETA = 2, E16_ROOTS = 4 };

template <typename CT>
struct Lev16View {
    const int64_t *off;
    const uint64_t *key;
    const CT *cnt;
};

// ---------------------------------------------------------------------------
// Bitstrings and counts
// ---------------------------------------------------------------------------
// length of the first root child word of the string s of len bits (0 if len = 0)
__device__ inline int first_word_len(uint32_t s, int len)
{
    int depth = 0;
    for (int i = 0; i < len; i++) {
        depth += ((s >> (len - 1 - i)) & 1u) ? 1 : -1;
        if (depth == 0) return i + 1;
    }
    return 0;
}

// The word w (lw bits) is not smaller than the word c (lc bits, lc = 0: no
// word). Both are primitive Dyck words, and a primitive Dyck word is never a
// proper prefix of another, so their common-length prefixes decide.
__device__ inline bool word_not_smaller(uint32_t w, int lw, uint32_t c, int lc)
{
    if (lc == 0) return true;
    const int m = min(lw, lc);
    return (w >> (lw - m)) >= (c >> (lc - m));
}

// beta_T: the number of root child words of T (string s, len bits) equal to
// the first one; children are in descending order, so equal ones lead.
__device__ inline uint32_t beta_of(uint32_t s, int len)
{
    int depth = 0, start = 0, flen = 0;
    uint32_t first = 0, b = 0;
    for (int i = 0; i < len; i++) {
        depth += ((s >> (len - 1 - i)) & 1u) ? 1 : -1;
        if (depth == 0) {
            const int l = i - start + 1;
            const uint32_t w = (s >> (len - 1 - i)) & ((1u << l) - 1u);
            if (flen == 0) { first = w; flen = l; b = 1; }
            else if (l == flen && w == first) b++;
            else break;
            start = i + 1;
        }
    }
    return b;
}

__device__ inline u128 mul_checked(u128 a, u128 b, bool &ovf)
{
    const uint64_t ah = hi64(a), bh = hi64(b);
    if (ah && bh) { ovf = true; return 0; }
    const u128 big = ah ? a : b;
    const uint64_t sm = ah ? lo64(b) : lo64(a);
    const u128 plo = (u128)lo64(big) * sm, phi = (u128)hi64(big) * sm;
    if (hi64(phi)) { ovf = true; return 0; }
    const u128 r = plo + (phi << 64);
    if (r < plo) ovf = true;
    return r;
}

// Unsigned 256-bit counts: four 64-bit words, least significant first.
struct U256 {
    uint64_t w[4];
};

// The arithmetic the kernels need, for either count type.
template <typename CT> struct Cnt;

template <> struct Cnt<u128> {
    static constexpr int words = 2;
    __device__ static u128 of(uint64_t x) { return x; }
    __device__ static bool zero(u128 a) { return a == 0; }
    __device__ static u128 add(u128 a, u128 b, bool &ovf)
    {
        const u128 t = a + b;
        if (t < a) ovf = true;
        return t;
    }
    __device__ static u128 mul(u128 a, u128 b, bool &ovf) { return mul_checked(a, b, ovf); }
    // a / d for 1 <= d < 2^32; inexact is set when d does not divide a
    __device__ static u128 div(u128 a, uint32_t d, bool &inexact)
    {
        const u128 q = div_small(a, d);
        if (q * d != a) inexact = true;
        return q;
    }
    __device__ static u128 shfl_up(u128 x, int d)
    {
        return mk128(__shfl_up((unsigned long long)lo64(x), d), __shfl_up((unsigned long long)hi64(x), d));
    }
    __device__ static uint64_t word(u128 x, int i) { return i == 0 ? lo64(x) : (i == 1 ? hi64(x) : 0); }
};

template <> struct Cnt<U256> {
    static constexpr int words = 4;
    __device__ static U256 of(uint64_t x)
    {
        U256 r = {{x, 0, 0, 0}};
        return r;
    }
    __device__ static bool zero(const U256 &a) { return !(a.w[0] | a.w[1] | a.w[2] | a.w[3]); }
    __device__ static U256 add(const U256 &a, const U256 &b, bool &ovf)
    {
        U256 r;
        uint64_t c = 0;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint64_t t = a.w[i] + b.w[i], u = t + c;
            c = (t < a.w[i] ? 1u : 0u) + (u < t ? 1u : 0u);
            r.w[i] = u;
        }
        if (c) ovf = true;
        return r;
    }
    // schoolbook on 64-bit words; any partial product above word 3 overflows
    __device__ static U256 mul(const U256 &a, const U256 &b, bool &ovf)
    {
        U256 r = {{0, 0, 0, 0}};
#pragma unroll
        for (int i = 0; i < 4; i++) {
            if (!a.w[i]) continue;
            uint64_t carry = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if (i + j >= 4) {
                    if (b.w[j]) ovf = true;
                    continue;
                }
                const u128 t = (u128)a.w[i] * b.w[j] + r.w[i + j] + carry;
                r.w[i + j] = lo64(t);
                carry = hi64(t);
            }
            if (carry) ovf = true;
        }
        return r;
    }
    // long division by 32-bit halves of the words, most significant first
    __device__ static U256 div(const U256 &a, uint32_t d, bool &inexact)
    {
        U256 q;
        uint64_t r = 0;
#pragma unroll
        for (int i = 3; i >= 0; i--) {
            uint64_t t = (r << 32) | (a.w[i] >> 32);
            const uint64_t qh = t / d;
            r = t % d;
            t = (r << 32) | (a.w[i] & 0xffffffffu);
            const uint64_t ql = t / d;
            r = t % d;
            q.w[i] = (qh << 32) | ql;
        }
        if (r) inexact = true;
        return q;
    }
    __device__ static U256 shfl_up(const U256 &x, int d)
    {
        U256 r;
#pragma unroll
        for (int i = 0; i < 4; i++) r.w[i] = __shfl_up((unsigned long long)x.w[i], d);
        return r;
    }
    __device__ static uint64_t word(const U256 &x, int i) { return x.w[i]; }
};

__device__ inline int binom_small(int n, int r)
{
    if (r < 0 || r > n) return 0;
    int b = 1;
    for (int i = 1; i <= r; i++) b = b * (n - r + i) / i;
    return b;
}

// next integer with the same number of set bits (Gosper)
__device__ inline uint32_t next_comb(uint32_t x)
{
    const uint32_t c = x & (0u - x), r = x + c;
    return (((r ^ x) >> 2) >> __builtin_ctz(c)) | r;
}

// the bits of idx placed on the set bits of mask, lowest first
__device__ inline uint32_t deposit(uint32_t idx, uint32_t mask)
{
    uint32_t out = 0;
    for (int i = 0; mask; mask &= mask - 1u, i++)
        if ((idx >> i) & 1u) out |= mask & (0u - mask);
    return out;
}

// one slot per active lane, in lane order, from the wave's counter in LDS
__device__ inline uint64_t wave_reserve(uint64_t *ctr)
{
    const uint64_t m = __ballot(1);
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint64_t base = 0;
    if (lane_id() == leader) base = atomicAdd((unsigned long long *)ctr, (unsigned long long)__popcll(m));
    base = shfl64(base, leader);
    return base + (uint64_t)__popcll(m & lanemask_lt());
}

// ---------------------------------------------------------------------------
// Level 1 and the neighbour sums
// ---------------------------------------------------------------------------
template <typename CT>
__global__ void k16_level1(const uint8_t *colors, int64_t n, int64_t *off, uint64_t *key, CT *cnt)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v <= n) off[v] = v;
    if (v < n) {
        key[v] = 1ull << colors[v];
        cnt[v] = Cnt<CT>::of(1);
    }
}

template <typename CT>
struct NbrArgs {
    const int64_t *row_ptr;
    const int32_t *col_idx;
    const uint8_t *colors;
    int64_t v0, v1;             // vertices [v0, v1)
    Lev16View<CT> X;            // level j
    int j, KB;                  // S_j sort key: C << 2(j-1) | s, KB bits
    int64_t *tnum;              // count: terms of v (written at tnum[v])
    const int64_t *toff;        // emit: exclusive term offsets over all vertices
    uint64_t *tkey;             // emit: (v - v0) << KB | sort key, at toff[v] - toff[v0] + i
    CT *tcnt;
};

// S_j(v): the entries of the neighbours' level-j records whose colour set
// avoids c_v. One wave per vertex; the neighbours are taken 64 at a time and
// their records walked as one flat range (entry f lies in the last record
// starting at or before f).
template <bool EMIT, typename CT>
__global__ __launch_bounds__(BLOCK) void k16_nbr(NbrArgs<CT> A)
{
    __shared__ int64_t seg_a[WPB][WAVE];
    __shared__ int64_t seg_p[WPB][WAVE];
    const int w = threadIdx.x / WAVE, lane = lane_id();
    const int64_t nw = (int64_t)gridDim.x * WPB;
    const int sb = 2 * (A.j - 1);
    for (int64_t v = A.v0 + (int64_t)blockIdx.x * WPB + w; v < A.v1; v += nw) {
        const uint32_t cbit = 1u << A.colors[v];
        const int64_t r0 = A.row_ptr[v], r1 = A.row_ptr[v + 1];
        uint64_t kept = 0;
        int64_t pos = EMIT ? A.toff[v] - A.toff[A.v0] : 0;
        const uint64_t vl = (uint64_t)(v - A.v0) << A.KB;
        for (int64_t r = r0; r < r1; r += WAVE) {
            const int nn = (int)min<int64_t>(WAVE, r1 - r);
            int64_t a = 0, len = 0;
            if (lane < nn) {
                const int32_t u = A.col_idx[r + lane];
                a = A.X.off[u];
                len = A.X.off[u + 1] - a;
            }
            const int64_t incl = (int64_t)wave_incl_scan64((uint64_t)len);
            const int64_t total = (int64_t)last_lane64((uint64_t)incl);
            seg_a[w][lane] = a;
            seg_p[w][lane] = incl - len;
            __builtin_amdgcn_wave_barrier();
            for (int64_t f0 = 0; f0 < total; f0 += WAVE) {
                const int64_t f = f0 + lane;
                bool keep = false;
                uint64_t key = 0;
                int64_t e = 0;
                if (f < total) {
                    int lo = 0, hi = nn - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (seg_p[w][mid] <= f) lo = mid; else hi = mid - 1;
                    }
                    e = seg_a[w][lo] + (f - seg_p[w][lo]);
                    key = A.X.key[e];
                    keep = !((uint32_t)key & cbit);
                }
                if (EMIT) {
                    const uint64_t m = __ballot(keep);
                    if (keep) {
                        const int64_t q = pos + __popcll(m & lanemask_lt());
                        const uint64_t C = key & 0xffffu, s = key >> 16;
                        A.tkey[q] = vl | (C << sb) | s;
                        A.tcnt[q] = A.X.cnt[e];
                    }
                    pos += __popcll(m);
                } else {
                    kept += keep ? 1u : 0u;
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (!EMIT) {
            const uint64_t t = wave_sum64(kept);
            if (lane == 0) A.tnum[v] = (int64_t)t;
        }
    }
}

// ---------------------------------------------------------------------------
// Eq. (1): the products of a level
// ---------------------------------------------------------------------------
template <typename CT>
struct CombArgs {
    const uint8_t *colors;
    int64_t v0, v1;
    int h, k, KB;               // X_h sort key: s_T << k | C, KB bits
    int zero_rooting;           // level k only at colour-0 vertices
    Lev16View<CT> X[K16];       // X[hp], hp = 1..h-1
    Lev16View<CT> S[K16];       // S[j], j = 1..h-1
    int64_t *tnum;
    const int64_t *toff;
    uint64_t *tkey;
    CT *tcnt;
    int *err;
};

// One wave per vertex v, one lane per own entry (T', C') of each level hp < h:
// the sums (T'', D) of S_{h-hp}(v) with D disjoint from C' whose word may
// lead T'. Three ways to find them, chosen per (v, hp) for the whole wave:
//  * a short record is walked entry by entry (every lane reads the same entry);
//  * otherwise each lane lists the (h-hp)-subsets D of its free colours and
//    looks each up in a directory of the record in LDS, indexed by the colex
//    rank of D among the (h-hp)-subsets of the k-1 colours other than c_v (the
//    record is sorted by D, and colex order of equal-size sets is their
//    numeric order, so each D's sums are one range);
//  * when that directory would exceed DIR_MAX entries, by binary search.
constexpr int DIR_MAX = 512;

template <bool EMIT, typename CT>
__global__ __launch_bounds__(BLOCK) void k16_comb(CombArgs<CT> A)
{
    __shared__ uint64_t ctr[WPB];
    __shared__ uint32_t dir_st[WPB][DIR_MAX];
    __shared__ uint32_t dir_en[WPB][DIR_MAX];
    __shared__ uint16_t binom_t[K16][K16 + 1];     // binom(p, q), p < 16, q <= 16
    // the lanes' own entries and ranges for the directory path (one set per wave)
    __shared__ uint32_t own_sp[WPB][WAVE], own_c1[WPB][WAVE], own_lc[WPB][WAVE], own_cd[WPB][WAVE];
    __shared__ uint32_t own_st[WPB][WAVE], own_ex[WPB][WAVE];
    __shared__ CT own_cx[WPB][WAVE];
    for (int q = threadIdx.x; q < K16 * (K16 + 1); q += BLOCK) {
        const int pp = q / (K16 + 1), qq = q % (K16 + 1);
        binom_t[pp][qq] = (uint16_t)binom_small(pp, qq);
    }
    __syncthreads();
    const int w = threadIdx.x / WAVE, lane = lane_id();
    const int64_t nw = (int64_t)gridDim.x * WPB;
    const uint32_t full = (1u << A.k) - 1u;
    // colex rank of a set of j colours of the (k-1)-colour universe
    auto rank_of = [&](uint32_t Dc) {
        uint32_t r = 0;
        for (int t = 1; Dc; Dc &= Dc - 1u, t++) r += binom_t[__builtin_ctz(Dc)][t];
        return r;
    };
    for (int64_t v = A.v0 + (int64_t)blockIdx.x * WPB + w; v < A.v1; v += nw) {
        if (lane == 0) ctr[w] = 0;
        __builtin_amdgcn_wave_barrier();
        uint64_t nterms = 0;
        bool ovf = false;
        const int64_t base = EMIT ? A.toff[v] - A.toff[A.v0] : 0;
        const uint64_t vl = (uint64_t)(v - A.v0) << A.KB;
        const int cv = A.colors[v];
        const bool active = !(A.zero_rooting && A.h == A.k && cv != 0);
        for (int hp = 1; active && hp < A.h; hp++) {
            const int j = A.h - hp, lp = 2 * (hp - 1), sb = 2 * (j - 1), lw = 2 * j;
            const Lev16View<CT> X = A.X[hp], S = A.S[j];
            const int64_t xa = X.off[v], xb = X.off[v + 1], sa = S.off[v], se = S.off[v + 1];
            if (xa == xb || sa == se) continue;
            const uint32_t smask = (1u << sb) - 1u;
            const int64_t nb = se - sa;
            const int m = A.k - hp;
            const int nsub = binom_small(m, j), ndir = binom_small(A.k - 1, j);
            int lg = 1;
            while (((int64_t)1 << lg) < nb) lg++;
            const int mode = nb <= (int64_t)nsub * 4 ? 0 : (ndir <= DIR_MAX ? 1 : 2);   // walk, directory, search
            if (mode == 1) {
                for (int q = lane; q < ndir; q += WAVE) dir_st[w][q] = dir_en[w][q] = 0;
                __builtin_amdgcn_wave_barrier();
                uint32_t prevD = 0xffffffffu;
                for (int64_t e0 = sa; e0 < se; e0 += WAVE) {
                    const int64_t e = e0 + lane;
                    const uint32_t D = e < se ? (uint32_t)(S.key[e] >> sb) : 0xffffffffu;
                    uint32_t before = (uint32_t)shfl64(D, lane == 0 ? 0 : lane - 1);
                    if (lane == 0) before = prevD;
                    if (e < se && D != before) {
                        dir_st[w][rank_of(compress_out(D, cv))] = (uint32_t)(e - sa);
                        if (before != 0xffffffffu) dir_en[w][rank_of(compress_out(before, cv))] = (uint32_t)(e - sa);
                    }
                    prevD = (uint32_t)readlane64(D, WAVE - 1);
                }
                if (lane == 0) {
                    const uint32_t last = (uint32_t)(S.key[se - 1] >> sb);
                    dir_en[w][rank_of(compress_out(last, cv))] = (uint32_t)nb;
                }
                __builtin_amdgcn_wave_barrier();
            }
            if (mode == 1) {
                // directory path, one colour subset per lane at a time: the lanes'
                // ranges of sums are laid end to end and the wave takes 64 sums per
                // round, so the lanes stay together and slots come from one ballot
                for (int64_t x0 = xa; x0 < xb; x0 += WAVE) {
                    const int64_t x = x0 + lane;
                    const bool xv = x < xb;
                    uint32_t Cp = 0, sp = 0, c1 = 0, freec = 0;
                    int lc = 0;
                    CT cx = Cnt<CT>::of(0);
                    uint64_t pos = 0;
                    if (xv) {
                        const uint64_t kx = X.key[x];
                        Cp = (uint32_t)kx & 0xffffu;
                        sp = (uint32_t)(kx >> 16);
                        lc = first_word_len(sp, lp);
                        c1 = lc ? sp >> (lp - lc) : 0u;
                        cx = X.cnt[x];
                        freec = compress_out(full & ~Cp, cv);
                        int t = 0;
                        for (uint32_t f = freec; f; f &= f - 1u, t++) pos |= (uint64_t)__builtin_ctz(f) << (4 * t);
                    }
                    own_sp[w][lane] = sp;
                    own_c1[w][lane] = c1;
                    own_lc[w][lane] = (uint32_t)lc;
                    own_cx[w][lane] = cx;
                    for (uint32_t idx = (1u << j) - 1u; idx < (1u << m); idx = next_comb(idx)) {
                        uint32_t st = 0, cntd = 0, D = 0;
                        if (xv) {
                            uint32_t Dc = 0, r = 0;
                            int t = 1;
                            for (uint32_t b = idx; b; b &= b - 1u, t++) {
                                const int p = (int)((pos >> (4 * __builtin_ctz(b))) & 15u);
                                Dc |= 1u << p;
                                r += binom_t[p][t];
                            }
                            st = dir_st[w][r];
                            cntd = dir_en[w][r] - st;
                            D = expand_in(Dc, cv);
                        }
                        const uint32_t incl = wave_incl_scan32(cntd);
                        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, WAVE - 1);
                        if (total == 0) continue;
                        own_st[w][lane] = st;
                        own_ex[w][lane] = incl - cntd;
                        own_cd[w][lane] = Cp | D;
                        __builtin_amdgcn_wave_barrier();
                        for (uint32_t f0 = 0; f0 < total; f0 += WAVE) {
                            const uint32_t f = f0 + lane;
                            bool keep = false;
                            uint64_t okey = 0;
                            CT prod = Cnt<CT>::of(0);
                            if (f < total) {
                                int lo = 0, hi = WAVE - 1;   // the last lane whose range starts at or before f
                                while (lo < hi) {
                                    const int mid = (lo + hi + 1) >> 1;
                                    if (own_ex[w][mid] <= f) lo = mid; else hi = mid - 1;
                                }
                                const int64_t e = sa + own_st[w][lo] + (f - own_ex[w][lo]);
                                const uint64_t ks = S.key[e];
                                const uint32_t wd = (1u << (lw - 1)) | (((uint32_t)ks & smask) << 1);
                                if (word_not_smaller(wd, lw, own_c1[w][lo], (int)own_lc[w][lo])) {
                                    keep = true;
                                    if (EMIT) {
                                        const uint64_t sT = ((uint64_t)wd << lp) | own_sp[w][lo];
                                        okey = vl | (sT << A.k) | (uint64_t)own_cd[w][lo];
                                        prod = Cnt<CT>::mul(own_cx[w][lo], S.cnt[e], ovf);
                                    }
                                }
                            }
                            if (EMIT) {
                                const uint64_t mk = __ballot(keep);
                                const uint64_t b0 = ctr[w];
                                if (keep) {
                                    const uint64_t q = (uint64_t)base + b0 + (uint64_t)__popcll(mk & lanemask_lt());
                                    A.tkey[q] = okey;
                                    A.tcnt[q] = prod;
                                }
                                __builtin_amdgcn_wave_barrier();
                                if (lane == 0) ctr[w] = b0 + (uint64_t)__popcll(mk);
                                __builtin_amdgcn_wave_barrier();
                            } else {
                                nterms += keep ? 1u : 0u;
                            }
                        }
                        __builtin_amdgcn_wave_barrier();
                    }
                }
                __builtin_amdgcn_wave_barrier();
                continue;
            }
            for (int64_t x = xa + lane; x < xb; x += WAVE) {
                const uint64_t kx = X.key[x];
                const uint32_t Cp = (uint32_t)kx & 0xffffu, sp = (uint32_t)(kx >> 16);
                const int lc = first_word_len(sp, lp);
                const uint32_t c1 = lc ? sp >> (lp - lc) : 0u;
                const CT cx = X.cnt[x];
                auto term = [&](int64_t e, uint32_t D) {
                    const uint64_t ks = S.key[e];
                    const uint32_t wd = (1u << (lw - 1)) | (((uint32_t)ks & smask) << 1);
                    if (!word_not_smaller(wd, lw, c1, lc)) return;
                    if (!EMIT) { nterms++; return; }
                    const uint64_t q = (uint64_t)base + wave_reserve(&ctr[w]);
                    const uint64_t sT = ((uint64_t)wd << lp) | sp;
                    A.tkey[q] = vl | (sT << A.k) | (uint64_t)(Cp | D);
                    A.tcnt[q] = Cnt<CT>::mul(cx, S.cnt[e], ovf);
                };
                if (mode == 0) {
                    for (int64_t e = sa; e < se; e++) {
                        const uint32_t D = (uint32_t)(S.key[e] >> sb);
                        if (!(D & Cp)) term(e, D);
                    }
                } else {
                    const uint32_t freec = full & ~Cp;
                    for (uint32_t idx = (1u << j) - 1u; idx < (1u << m); idx = next_comb(idx)) {
                        const uint32_t D = deposit(idx, freec);
                        const uint64_t lo_key = (uint64_t)D << sb;
                        int64_t lo = sa, hi = se;
                        while (lo < hi) {
                            const int64_t mid = (lo + hi) >> 1;
                            if (S.key[mid] < lo_key) lo = mid + 1; else hi = mid;
                        }
                        for (int64_t e = lo; e < se && (uint32_t)(S.key[e] >> sb) == D; e++) term(e, D);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (EMIT) {
            if (ovf) atomicOr(A.err, E16_OVERFLOW);
        } else {
            const uint64_t t = wave_sum64(nterms);
            if (lane == 0) A.tnum[v] = (int64_t)t;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of uint64 arrays (blocks of SCAN_TILE, then the block sums)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k16_scan_tiles(uint64_t *d, int64_t N, uint64_t *tile_sums)
{
    __shared__ uint64_t wsum[WPB];
    const int64_t t0 = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint64_t x[SCAN_ITEMS], s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        x[i] = t0 + i < N ? d[t0 + i] : 0;
        s += x[i];
    }
    const int w = threadIdx.x / WAVE, lane = lane_id();
    const uint64_t incl = wave_incl_scan64(s);
    if (lane == WAVE - 1) wsum[w] = incl;
    __syncthreads();
    uint64_t before = incl - s;
    for (int i = 0; i < w; i++) before += wsum[i];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        if (t0 + i < N) d[t0 + i] = before;
        before += x[i];
    }
    if (threadIdx.x == BLOCK - 1) tile_sums[blockIdx.x] = before;
}

__global__ void k16_scan_add(uint64_t *d, int64_t N, const uint64_t *tile_off)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) d[i] += tile_off[i / SCAN_TILE];
}

// ---------------------------------------------------------------------------
// Radix sort of (64-bit word, uint32 index) pairs, RADIX_BITS bits per pass
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k16_hist(const uint64_t *keys, int64_t N, int shift, uint64_t *hist,
                                                  int64_t nblocks)
{
    __shared__ uint32_t c[RADIX];
    for (int q = threadIdx.x; q < RADIX; q += BLOCK) c[q] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * SORT_TILE;
#pragma unroll 4
    for (int it = 0; it < SORT_ITEMS; it++) {
        const int64_t i = t0 + it * BLOCK + threadIdx.x;
        if (i < N) atomicAdd(&c[(keys[i] >> shift) & (RADIX - 1)], 1u);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < RADIX; q += BLOCK) hist[(int64_t)q * nblocks + blockIdx.x] = c[q];
}

// Stable scatter. Each wave owns a contiguous quarter of the tile (its items
// in index order), so an element's rank among the tile's elements of its digit
// is: the elements of that digit in earlier waves' quarters, plus those in the
// wave's earlier items (a per-wave count in LDS, kept by the wave alone), plus
// the earlier lanes of its item with that digit (one ballot per digit bit).
// off[d * nblocks + b] is where digit d of block b starts. Two block barriers
// per tile: after the counts, and after their running sum over the waves.
__global__ __launch_bounds__(BLOCK) void k16_scatter(const uint64_t *kin, const uint32_t *pin, uint64_t *kout,
                                                     uint32_t *pout, int64_t N, int shift, const uint64_t *off,
                                                     int64_t nblocks)
{
    __shared__ uint32_t wc[WPB][RADIX];   // per wave: elements of each digit so far, then the waves before
    const int w = threadIdx.x / WAVE, lane = lane_id();
    for (int q = threadIdx.x; q < WPB * RADIX; q += BLOCK) wc[q / RADIX][q % RADIX] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE + (int64_t)w * (SORT_ITEMS * WAVE);
    uint64_t key[SORT_ITEMS];
    uint32_t p[SORT_ITEMS], rank[SORT_ITEMS];
#pragma unroll
    for (int it = 0; it < SORT_ITEMS; it++) {
        const int64_t i = base + it * WAVE + lane;
        key[it] = i < N ? kin[i] : 0;
        p[it] = i < N ? (pin ? pin[i] : (uint32_t)i) : 0;
    }
#pragma unroll
    for (int it = 0; it < SORT_ITEMS; it++) {
        const bool valid = base + it * WAVE + lane < N;
        const uint32_t d = (uint32_t)(key[it] >> shift) & (RADIX - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RADIX_BITS; b++) {
            const uint64_t ones = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? ones : ~ones;
        }
        const uint64_t below = peers & lanemask_lt();
        const uint32_t cur = valid ? wc[w][d] : 0u;
        rank[it] = cur + (uint32_t)__popcll(below);
        if (valid && below == 0) wc[w][d] = cur + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < RADIX; q += BLOCK) {
        uint32_t run = 0;
        for (int x = 0; x < WPB; x++) {
            const uint32_t c = wc[x][q];
            wc[x][q] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < SORT_ITEMS; it++) {
        if (base + it * WAVE + lane >= N) continue;
        const uint32_t d = (uint32_t)(key[it] >> shift) & (RADIX - 1);
        const uint64_t pos = off[(int64_t)d * nblocks + blockIdx.x] + wc[w][d] + rank[it];
        kout[pos] = key[it];
        pout[pos] = p[it];
    }
}

// ---------------------------------------------------------------------------
// Aggregation of sorted terms
// ---------------------------------------------------------------------------
constexpr int RUN_ITEMS = 4;                       // sorted terms per thread of the run sums
constexpr int RUN_TILE = BLOCK * RUN_ITEMS;         // sorted terms per block

// Run heads (first terms of runs of equal words) per block of RUN_TILE sorted terms.
__global__ __launch_bounds__(BLOCK) void k16_heads(const uint64_t *keys, int64_t N, uint64_t *bcount)
{
    __shared__ uint32_t wsum[WPB];
    const int64_t i0 = (int64_t)blockIdx.x * RUN_TILE + (int64_t)threadIdx.x * RUN_ITEMS;
    uint32_t c = 0;
    uint64_t prev = i0 > 0 && i0 < N ? keys[i0 - 1] : 0;
#pragma unroll
    for (int j = 0; j < RUN_ITEMS; j++) {
        const int64_t i = i0 + j;
        if (i < N) {
            const uint64_t kw = keys[i];
            if (i == 0 || kw != prev) c++;
            prev = kw;
        }
    }
    const uint32_t t = (uint32_t)wave_sum64(c);
    if (lane_id() == 0) wsum[threadIdx.x / WAVE] = t;
    __syncthreads();
    if (threadIdx.x == 0) bcount[blockIdx.x] = (uint64_t)wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// x += v at p (two 64-bit atomics, the low word's carry passed on); true when
// the 128-bit sum wraps
__device__ inline bool atomic_add128(u128 *p, u128 v)
{
    unsigned long long *w = (unsigned long long *)p;
    const unsigned long long lo = lo64(v), hi = hi64(v);
    const unsigned long long old = atomicAdd(&w[0], lo);
    const unsigned long long add_hi = hi + (old + lo < old ? 1ull : 0ull);
    bool wrap = add_hi < hi;
    if (add_hi) {
        const unsigned long long oh = atomicAdd(&w[1], add_hi);
        if (oh + add_hi < oh) wrap = true;
    }
    return wrap;
}

// the same for four words: each word's carry (out of the add, or out of the
// atomic) goes into the next one
__device__ inline bool atomic_add256(U256 *p, const U256 &v)
{
    unsigned long long *w = (unsigned long long *)p;
    unsigned long long carry = 0;
    for (int i = 0; i < 4; i++) {
        const unsigned long long add = v.w[i] + carry;
        carry = add < v.w[i] ? 1ull : 0ull;
        if (add) {
            const unsigned long long old = atomicAdd(&w[i], add);
            if (old + add < old) carry++;
        }
    }
    return carry != 0;
}
__device__ inline bool atomic_addc(u128 *p, u128 v) { return atomic_add128(p, v); }
__device__ inline bool atomic_addc(U256 *p, const U256 &v) { return atomic_add256(p, v); }

template <typename CT>
struct RunArgs {
    const uint64_t *keys;       // sorted words
    const uint32_t *perm;       // term index of each sorted word
    const CT *tcnt;
    const uint64_t *bhead;      // exclusive scan of the blocks' run heads
    int64_t N;
    int KB;
    int64_t v0;
    CT *ocnt;                   // [U] sums, zero on entry
    uint64_t *oword;            // [U] the run's word
    int64_t *vcount;            // [n] entries per vertex
    int *err;
};

// Sums of the runs of equal words. Each thread takes RUN_ITEMS consecutive
// sorted terms and fetches their counts (independent loads); it sums the
// elements after its last run head, the wave passes those partial sums on by a
// segmented scan over lanes, and the last element of each run piece writes the
// piece's sum: a run that lies wholly in the wave's range is stored, a piece of
// a longer run is added to the run's output atomically.
template <typename CT>
__global__ __launch_bounds__(BLOCK) void k16_runsum(RunArgs<CT> A)
{
    __shared__ uint32_t wheads[WPB];
    const int lane = lane_id(), wv = threadIdx.x / WAVE;
    const int64_t i0 = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * RUN_ITEMS;
    uint64_t word[RUN_ITEMS], o[RUN_ITEMS];
    CT val[RUN_ITEMS];
    bool head[RUN_ITEMS], valid[RUN_ITEMS];
    uint64_t prev = i0 > 0 && i0 < A.N ? A.keys[i0 - 1] : 0;
#pragma unroll
    for (int j = 0; j < RUN_ITEMS; j++) {
        const int64_t i = i0 + j;
        valid[j] = i < A.N;
        word[j] = valid[j] ? A.keys[i] : 0;
        head[j] = valid[j] && (i == 0 || (j == 0 ? prev : word[j - 1]) != word[j]);
    }
#pragma unroll
    for (int j = 0; j < RUN_ITEMS; j++) {
        const int64_t i = i0 + j;
        val[j] = valid[j] ? A.tcnt[A.perm[i]] : Cnt<CT>::of(0);
    }
    // output index of each term's run: the heads before it, minus one when it is
    // not a head itself (heads of earlier blocks, earlier waves, earlier lanes,
    // then this thread's own)
    uint32_t nh = 0;
#pragma unroll
    for (int j = 0; j < RUN_ITEMS; j++) nh += head[j] ? 1u : 0u;
    const uint32_t hincl = wave_incl_scan32(nh);
    if (lane == WAVE - 1) wheads[wv] = hincl;
    __syncthreads();
    uint64_t before = A.bhead[blockIdx.x] + (hincl - nh);
    for (int q = 0; q < wv; q++) before += wheads[q];
#pragma unroll
    for (int j = 0; j < RUN_ITEMS; j++) {
        before += head[j] ? 1u : 0u;
        o[j] = valid[j] ? before - 1u : 0u;
    }
    bool wrap = false, any = false;
    CT tail = Cnt<CT>::of(0);   // this thread's elements after its last head (all of them without one)
#pragma unroll
    for (int j = 0; j < RUN_ITEMS; j++) {
        if (head[j]) {
            tail = val[j];
            any = true;
        } else {
            tail = Cnt<CT>::add(tail, val[j], wrap);
        }
    }
    // inclusive segmented scan of (tail, any) over the lanes
    CT c = tail;
    bool f = any;
    for (int d = 1; d < WAVE; d <<= 1) {
        const CT pv = Cnt<CT>::shfl_up(c, d);
        const bool pf = __shfl_up((int)f, d) != 0;
        if (lane >= d) {
            if (!f) c = Cnt<CT>::add(c, pv, wrap);
            f = f || pf;
        }
    }
    // what the lanes before this one carry into its first run, and whether that
    // run's head lies in the wave's range
    CT run = Cnt<CT>::shfl_up(c, 1);
    bool seen = __shfl_up((int)f, 1) != 0;
    if (lane == 0) {
        run = Cnt<CT>::of(0);
        seen = false;
    }
    const bool next_lane_starts = __shfl_down((int)(head[0] || !valid[0]), 1) != 0;
#pragma unroll
    for (int j = 0; j < RUN_ITEMS; j++) {
        if (!valid[j]) break;
        if (head[j]) {
            run = val[j];
            seen = true;
        } else {
            run = Cnt<CT>::add(run, val[j], wrap);
        }
        bool ends, piece_end;
        if (j < RUN_ITEMS - 1) {
            ends = piece_end = !valid[j + 1] || head[j + 1];
        } else if (lane < WAVE - 1) {
            ends = piece_end = next_lane_starts;
        } else {
            piece_end = true;
            ends = i0 + j + 1 >= A.N || A.keys[i0 + j + 1] != word[j];
        }
        if (!piece_end) continue;
        if (seen && ends) A.ocnt[o[j]] = run;
        else wrap |= atomic_addc(&A.ocnt[o[j]], run);
    }
#pragma unroll
    for (int j = 0; j < RUN_ITEMS; j++)
        if (head[j]) {
            A.oword[o[j]] = word[j];
            atomicAdd((unsigned long long *)&A.vcount[A.v0 + (int64_t)(word[j] >> A.KB)], 1ull);
        }
    if (wrap) atomicOr(A.err, E16_OVERFLOW);
}

// The run words become keys; for X_h each sum is divided by beta_T.
template <typename CT>
__global__ void k16_finish(uint64_t *okey, CT *ocnt, int64_t U, int KB, int k, int hlen, int x_level, int *err)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= U) return;
    const uint64_t sk = okey[o] & ((1ull << KB) - 1ull);
    if (!x_level) {
        okey[o] = sk;
        return;
    }
    const uint32_t s = (uint32_t)(sk >> k), C = (uint32_t)sk & ((1u << k) - 1u);
    const uint32_t b = beta_of(s, hlen);
    if (b > 1) {
        bool inexact = false;
        ocnt[o] = Cnt<CT>::div(ocnt[o], b, inexact);
        if (inexact) atomicOr(err, E16_BETA);
    }
    okey[o] = ((uint64_t)s << 16) | C;
}

// ---------------------------------------------------------------------------
// Totals and export
// ---------------------------------------------------------------------------
// per-block checked sums of cnt[0, N) into part[block]
template <typename CT>
__global__ __launch_bounds__(BLOCK) void k16_sum(const CT *cnt, int64_t N, CT *part, int *err)
{
    __shared__ CT ws[BLOCK];
    CT s = Cnt<CT>::of(0);
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLOCK)
        s = Cnt<CT>::add(s, cnt[i], bad);
    ws[threadIdx.x] = s;
    __syncthreads();
    for (int st = BLOCK / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) ws[threadIdx.x] = Cnt<CT>::add(ws[threadIdx.x], ws[threadIdx.x + st], bad);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = ws[0];
    if (bad) atomicOr(err, E16_OVERFLOW);
}

// t = the sum of the level-k counts (divided by k when every vertex is a root),
// as four words
template <typename CT>
__global__ void k16_total(const CT *part, int nparts, int divide_by, uint64_t *out, int *err)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    CT s = Cnt<CT>::of(0);
    bool ovf = false, inexact = false;
    for (int i = 0; i < nparts; i++) s = Cnt<CT>::add(s, part[i], ovf);
    if (divide_by > 1) s = Cnt<CT>::div(s, (uint32_t)divide_by, inexact);
    if (ovf) atomicOr(err, E16_OVERFLOW);
    if (inexact) atomicOr(err, E16_ROOTS);
    for (int i = 0; i < 4; i++) out[i] = Cnt<CT>::word(s, i);
}

// counts as nwords words each (the count's own words, then zeros)
template <typename CT>
__global__ void k16_words(const CT *cnt, int64_t N, uint64_t *out, int nwords)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) {
        const CT c = cnt[i];
        for (int q = 0; q < nwords; q++) out[i * nwords + q] = Cnt<CT>::word(c, q);
    }
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }
inline unsigned wave_grid(int64_t nv) { return (unsigned)std::min<int64_t>(std::max<int64_t>(1, (nv + WPB - 1) / WPB), 65536); }

} // namespace

// ---------------------------------------------------------------------------
// The table
// ---------------------------------------------------------------------------
struct Lev16 {
    int64_t *off = nullptr;
    uint64_t *key = nullptr;
    void *cnt = nullptr;        // u128[nnz] or U256[nnz], by the table's width
    int64_t nnz = 0;
    template <typename CT> Lev16View<CT> view() const { return {off, key, (const CT *)cnt}; }
};

struct scc16_table {
    int k = 0, rooting = SCC_ROOT_ZERO;
    int64_t n = 0, nnz_g = 0, chunk_terms = DEFAULT_CHUNK_TERMS;
    const int64_t *row_ptr = nullptr;
    const int32_t *col_idx = nullptr;
    const uint8_t *colors = nullptr;
    hipStream_t stream = nullptr;
    DevMem mem;
    std::vector<void *> owned;      // device blocks held by the table
    Lev16 X[K16 + 1];
    int count_bits = 128;           // width of every stored count: 128 or 256
    uint64_t t[4] = {0, 0, 0, 0};
    scc16_table_info info{};
    int64_t live = 0;               // device bytes of the build at this moment (for peak_bytes)

    void *hold(size_t bytes)
    {
        void *p = mem.get(bytes);
        if (p) owned.push_back(p);
        return p;
    }
    ~scc16_table()
    {
        if (!owned.empty()) (void)hipStreamSynchronize(stream);
        for (void *p : owned) mem.put(p);
    }
};

namespace {

// Device blocks of one build step, returned to the allocator on scope exit.
struct Scratch {
    scc16_table *T;
    std::vector<std::pair<void *, size_t>> blocks;
    explicit Scratch(scc16_table *t) : T(t) {}
    void *get(size_t bytes)
    {
        void *p = T->mem.get(bytes);
        if (p) {
            blocks.push_back({p, bytes});
            T->live += (int64_t)bytes;
            T->info.peak_bytes = std::max(T->info.peak_bytes, T->live);
        }
        return p;
    }
    void put(void *p)
    {
        for (size_t i = 0; i < blocks.size(); i++)
            if (blocks[i].first == p) {
                T->mem.put(p);
                T->live -= (int64_t)blocks[i].second;
                blocks.erase(blocks.begin() + (long)i);
                return;
            }
    }
    ~Scratch()
    {
        for (auto &b : blocks) {
            T->mem.put(b.first);
            T->live -= (int64_t)b.second;
        }
    }
};

// in-place exclusive scan of d[0, N); the total goes to *total (device)
scc_status scan_u64(scc16_table *T, uint64_t *d, int64_t N, uint64_t *total)
{
    if (N <= 0) {
        HIP_TRY(hipMemsetAsync(total, 0, 8, T->stream));
        return SCC_OK;
    }
    const int64_t nb = (N + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL(k16_scan_tiles, dim3(1), dim3(BLOCK), 0, T->stream, d, N, total);
        return SCC_OK;
    }
    Scratch sc(T);
    uint64_t *sums = (uint64_t *)sc.get((size_t)nb * 8);
    if (!sums) return set_error(SCC_ENOMEM, "scan");
    hipLaunchKernelGGL(k16_scan_tiles, dim3((unsigned)nb), dim3(BLOCK), 0, T->stream, d, N, sums);
    scc_status s = scan_u64(T, sums, nb, total);
    if (s) return s;
    hipLaunchKernelGGL(k16_scan_add, dim3(blocks_for(N, 256)), dim3(256), 0, T->stream, d, N, sums);
    return SCC_OK;
}

// Sorts keys[0, N) (bits [0, bits) significant) carrying a uint32 index that
// starts as the identity; on return *keys and *perm point at the sorted data
// (one of the two buffers each).
scc_status radix_sort(scc16_table *T, uint64_t **keys, uint64_t *keys_alt, uint32_t **perm, uint32_t *perm_alt,
                      int64_t N, int bits, uint64_t *hist, uint64_t *total, double &bytes)
{
    if (bits <= 0) return set_error(SCC_EINVAL, "radix sort without key bits");
    const int64_t nb = (N + SORT_TILE - 1) / SORT_TILE;
    uint64_t *kin = *keys, *kout = keys_alt;
    uint32_t *pin = nullptr, *pout = *perm, *pspare = perm_alt;
    for (int shift = 0; shift < bits; shift += RADIX_BITS) {
        hipLaunchKernelGGL(k16_hist, dim3((unsigned)nb), dim3(BLOCK), 0, T->stream, kin, N, shift, hist, nb);
        scc_status s = scan_u64(T, hist, nb * RADIX, total);
        if (s) return s;
        hipLaunchKernelGGL(k16_scatter, dim3((unsigned)nb), dim3(BLOCK), 0, T->stream, kin, pin, kout, pout, N, shift,
                           hist, nb);
        bytes += 32.0 * (double)N;
        std::swap(kin, kout);
        pin = pout;
        pout = (pout == *perm) ? pspare : *perm;
    }
    *keys = kin;
    *perm = pin;
    return SCC_OK;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() { (void)hipEventCreate(&a); (void)hipEventCreate(&b); }
    ~Timer() { if (a) (void)hipEventDestroy(a); if (b) (void)hipEventDestroy(b); }
    void start(hipStream_t s) { (void)hipEventRecord(a, s); }
    double stop(hipStream_t s)
    {
        float ms = 0;
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        (void)hipEventElapsedTime(&ms, a, b);
        return ms;
    }
};

// One level: x_level = 1 builds X_h from X_1..X_{h-1} and S_1..S_{h-1}
// (Eq. (1)); x_level = 0 builds S_h from X_h. `own` receives the result; its
// arrays are held by the table (X) or by `hold` (S, freed after the build).
template <typename CT>
scc_status build_pass(scc16_table *T, int x_level, int h, const Lev16 *S, Lev16 &out, std::vector<void *> &hold,
                      int64_t &terms_out, int64_t &chunks_out, double &sort_ms, double &sort_bytes)
{
    constexpr size_t CB = sizeof(CT);
    const int64_t n = T->n;
    const int k = T->k, KB = 2 * (h - 1) + k;
    Scratch sc(T);
    auto keep = [&](size_t bytes) -> void * {
        void *p = x_level ? T->hold(bytes) : T->mem.get(bytes);
        if (p && !x_level) hold.push_back(p);
        if (p) { T->live += (int64_t)bytes; T->info.peak_bytes = std::max(T->info.peak_bytes, T->live); }
        return p;
    };
    uint64_t *toff = (uint64_t *)sc.get((size_t)(n + 1) * 8);
    uint64_t *word = (uint64_t *)sc.get(64);
    int *err = (int *)sc.get(64);
    if (!toff || !word || !err) return set_error(SCC_ENOMEM, "level %d terms", h);
    HIP_TRY(hipMemsetAsync(toff, 0, (size_t)(n + 1) * 8, T->stream));
    HIP_TRY(hipMemsetAsync(err, 0, 4, T->stream));

    NbrArgs<CT> NA{};
    CombArgs<CT> CA{};
    if (x_level) {
        CA.colors = T->colors;
        CA.h = h;
        CA.k = k;
        CA.KB = KB;
        CA.zero_rooting = T->rooting == SCC_ROOT_ZERO;
        for (int q = 1; q < h; q++) {
            CA.X[q] = T->X[q].view<CT>();
            CA.S[q] = S[q].view<CT>();
        }
        CA.err = err;
        CA.tnum = (int64_t *)toff;
        CA.v0 = 0;
        CA.v1 = n;
        hipLaunchKernelGGL((k16_comb<false, CT>), dim3(wave_grid(n)), dim3(BLOCK), 0, T->stream, CA);
    } else {
        NA.row_ptr = T->row_ptr;
        NA.col_idx = T->col_idx;
        NA.colors = T->colors;
        NA.X = T->X[h].view<CT>();
        NA.j = h;
        NA.KB = KB;
        NA.tnum = (int64_t *)toff;
        NA.v0 = 0;
        NA.v1 = n;
        hipLaunchKernelGGL((k16_nbr<false, CT>), dim3(wave_grid(n)), dim3(BLOCK), 0, T->stream, NA);
    }
    HIP_TRY(hipGetLastError());
    scc_status s = scan_u64(T, toff, n + 1, word);
    if (s) return s;
    std::vector<int64_t> ht((size_t)n + 1);
    HIP_TRY(hipMemcpyAsync(ht.data(), toff, (size_t)(n + 1) * 8, hipMemcpyDeviceToHost, T->stream));
    HIP_TRY(hipStreamSynchronize(T->stream));
    terms_out = ht[(size_t)n];

    // vertex chunks: at most chunk_terms terms (a vertex with more is a chunk
    // of its own) and few enough vertices that (vertex, key) fits 64 bits
    const int vbits_max = std::min(64 - KB, 30);
    const int64_t vmax = (int64_t)1 << vbits_max;
    std::vector<std::pair<int64_t, int64_t>> chunks;
    int64_t nmax = 0;
    for (int64_t v = 0; v < n;) {
        int64_t v1 = v + 1;
        while (v1 < n && v1 - v < vmax && ht[(size_t)v1 + 1] - ht[(size_t)v] <= T->chunk_terms) v1++;
        const int64_t N = ht[(size_t)v1] - ht[(size_t)v];
        if (N > MAX_CHUNK_TERMS)
            return set_error(SCC_ENOMEM, "level %d: vertex %lld forms %lld terms (more than 2^31 - 1)", h,
                             (long long)v, (long long)N);
        if (N > 0) chunks.push_back({v, v1});
        nmax = std::max(nmax, N);
        v = v1;
    }
    chunks_out = (int64_t)chunks.size();

    out.off = (int64_t *)keep((size_t)(n + 1) * 8);
    if (!out.off) return set_error(SCC_ENOMEM, "level %d offsets", h);
    HIP_TRY(hipMemsetAsync(out.off, 0, (size_t)(n + 1) * 8, T->stream));
    std::vector<std::pair<uint64_t *, CT *>> parts;
    std::vector<int64_t> part_n;
    Scratch parts_mem(T);
    if (nmax > 0) {
        const int64_t nbs = (nmax + SORT_TILE - 1) / SORT_TILE;
        uint64_t *ka = (uint64_t *)sc.get((size_t)nmax * 8), *kb = (uint64_t *)sc.get((size_t)nmax * 8);
        uint32_t *pa = (uint32_t *)sc.get((size_t)nmax * 4), *pb = (uint32_t *)sc.get((size_t)nmax * 4);
        CT *tc = (CT *)sc.get((size_t)nmax * CB);
        uint64_t *flag = (uint64_t *)sc.get((size_t)((nmax + RUN_TILE - 1) / RUN_TILE + 1) * 8);
        uint64_t *hist = (uint64_t *)sc.get((size_t)nbs * RADIX * 8);
        if (!ka || !kb || !pa || !pb || !tc || !flag || !hist) return set_error(SCC_ENOMEM, "level %d sort", h);
        Timer tm;
        for (auto &c : chunks) {
            const int64_t v0 = c.first, v1 = c.second, N = ht[(size_t)v1] - ht[(size_t)v0];
            if (x_level) {
                CA.v0 = v0; CA.v1 = v1; CA.toff = (const int64_t *)toff; CA.tkey = ka; CA.tcnt = tc;
                hipLaunchKernelGGL((k16_comb<true, CT>), dim3(wave_grid(v1 - v0)), dim3(BLOCK), 0, T->stream, CA);
            } else {
                NA.v0 = v0; NA.v1 = v1; NA.toff = (const int64_t *)toff; NA.tkey = ka; NA.tcnt = tc;
                hipLaunchKernelGGL((k16_nbr<true, CT>), dim3(wave_grid(v1 - v0)), dim3(BLOCK), 0, T->stream, NA);
            }
            HIP_TRY(hipGetLastError());
            int vb = 0;
            while (((int64_t)1 << vb) < v1 - v0) vb++;
            uint64_t *keys = ka;
            uint32_t *perm = pa;
            tm.start(T->stream);
            s = radix_sort(T, &keys, kb, &perm, pb, N, KB + vb, hist, word, sort_bytes);
            if (s) return s;
            sort_ms += tm.stop(T->stream);
            const int64_t nrb = (N + RUN_TILE - 1) / RUN_TILE;
            hipLaunchKernelGGL(k16_heads, dim3((unsigned)nrb), dim3(BLOCK), 0, T->stream, keys, N, flag);
            s = scan_u64(T, flag, nrb, word);
            if (s) return s;
            uint64_t U = 0;
            HIP_TRY(hipMemcpyAsync(&U, word, 8, hipMemcpyDeviceToHost, T->stream));
            HIP_TRY(hipStreamSynchronize(T->stream));
            uint64_t *ok = (uint64_t *)parts_mem.get((size_t)U * 8);
            CT *oc = (CT *)parts_mem.get((size_t)U * CB);
            if (!ok || !oc) return set_error(SCC_ENOMEM, "level %d records", h);
            HIP_TRY(hipMemsetAsync(oc, 0, (size_t)U * CB, T->stream));
            RunArgs<CT> R{keys, perm, tc, flag, N, KB, v0, oc, ok, out.off, err};
            hipLaunchKernelGGL((k16_runsum<CT>), dim3((unsigned)nrb), dim3(BLOCK), 0, T->stream, R);
            hipLaunchKernelGGL((k16_finish<CT>), dim3(blocks_for((int64_t)U, 256)), dim3(256), 0, T->stream, ok, oc,
                               (int64_t)U, KB, k, 2 * (h - 1), x_level, err);
            HIP_TRY(hipGetLastError());
            parts.push_back({ok, oc});
            part_n.push_back((int64_t)U);
        }
    }
    int64_t nnz = 0;
    for (int64_t u : part_n) nnz += u;
    out.nnz = nnz;
    out.key = (uint64_t *)keep((size_t)nnz * 8);
    out.cnt = keep((size_t)nnz * CB);
    if (!out.key || !out.cnt) return set_error(SCC_ENOMEM, "level %d records", h);
    int64_t at = 0;
    for (size_t i = 0; i < parts.size(); i++) {
        if (part_n[i] == 0) continue;
        HIP_TRY(hipMemcpyAsync(out.key + at, parts[i].first, (size_t)part_n[i] * 8, hipMemcpyDeviceToDevice, T->stream));
        HIP_TRY(hipMemcpyAsync((CT *)out.cnt + at, parts[i].second, (size_t)part_n[i] * CB, hipMemcpyDeviceToDevice,
                               T->stream));
        at += part_n[i];
    }
    s = scan_u64(T, (uint64_t *)out.off, n + 1, word);
    if (s) return s;
    int herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, T->stream));
    HIP_TRY(hipStreamSynchronize(T->stream));
    if (herr & E16_OVERFLOW)
        return set_error(SCC_EOVERFLOW, "level %d: a count needs more than %d bits", h, (int)(8 * CB));
    if (herr) return set_error(SCC_EDEVICE, "level %d: internal check failed (%d)", h, herr);
    return SCC_OK;
}

template <typename CT>
scc_status build_all(scc16_table *T)
{
    constexpr size_t CB = sizeof(CT);
    const int64_t n = T->n;
    const int k = T->k;
    Lev16 S[K16 + 1];
    std::vector<void *> hold;
    struct Free {
        scc16_table *T;
        std::vector<void *> &h;
        ~Free() { for (void *p : h) T->mem.put(p); }
    } fr{T, hold};
    Timer all;
    all.start(T->stream);
    // level 1: one count of 1 per vertex at ({root}, {c_v})
    {
        Lev16 &L = T->X[1];
        L.off = (int64_t *)T->hold((size_t)(n + 1) * 8);
        L.key = (uint64_t *)T->hold((size_t)std::max<int64_t>(n, 1) * 8);
        L.cnt = T->hold((size_t)std::max<int64_t>(n, 1) * CB);
        if (!L.off || !L.key || !L.cnt) return set_error(SCC_ENOMEM, "level 1");
        T->live += (n + 1) * 8 + n * (int64_t)(8 + CB);
        hipLaunchKernelGGL((k16_level1<CT>), dim3(blocks_for(n + 1, 256)), dim3(256), 0, T->stream, T->colors, n, L.off,
                           L.key, (CT *)L.cnt);
        HIP_TRY(hipGetLastError());
        L.nnz = n;
    }
    for (int h = 1; h <= k; h++) {
        Timer tl;
        tl.start(T->stream);
        double sms = 0, sbytes = 0;
        if (h >= 2) {
            int64_t terms = 0, chunks = 0;
            scc_status s = build_pass<CT>(T, 1, h, S, T->X[h], hold, terms, chunks, sms, sbytes);
            if (s) return s;
            T->info.terms[h] = terms;
            T->info.chunks[h] = chunks;
        }
        if (h < k) {
            int64_t terms = 0, chunks = 0;
            scc_status s = build_pass<CT>(T, 0, h, S, S[h], hold, terms, chunks, sms, sbytes);
            if (s) return s;
            T->info.nbr_terms[h] = terms;
            T->info.sum_nnz[h] = S[h].nnz;
        }
        T->info.level_ms[h] = tl.stop(T->stream);
        T->info.sort_ms[h] = sms;
        T->info.sort_bytes[h] = sbytes;
        T->info.nnz[h] = T->X[h].nnz;
    }
    // t
    {
        Scratch sc(T);
        const int parts = 256;
        CT *part = (CT *)sc.get(parts * CB);
        uint64_t *tout = (uint64_t *)sc.get(64);
        int *err = (int *)sc.get(64);
        if (!part || !tout || !err) return set_error(SCC_ENOMEM, "totals");
        HIP_TRY(hipMemsetAsync(err, 0, 4, T->stream));
        hipLaunchKernelGGL((k16_sum<CT>), dim3(parts), dim3(BLOCK), 0, T->stream, (const CT *)T->X[k].cnt, T->X[k].nnz,
                           part, err);
        hipLaunchKernelGGL((k16_total<CT>), dim3(1), dim3(64), 0, T->stream, (const CT *)part, parts,
                           T->rooting == SCC_ROOT_ALL ? k : 1, tout, err);
        HIP_TRY(hipGetLastError());
        int herr = 0;
        HIP_TRY(hipMemcpyAsync(T->t, tout, 32, hipMemcpyDeviceToHost, T->stream));
        HIP_TRY(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, T->stream));
        HIP_TRY(hipStreamSynchronize(T->stream));
        if (herr & E16_OVERFLOW) return set_error(SCC_EOVERFLOW, "t needs more than %d bits", (int)(8 * CB));
        if (herr) return set_error(SCC_EDEVICE, "the level-k sum is not a multiple of k");
    }
    T->info.build_ms = all.stop(T->stream);
    return SCC_OK;
}

} // namespace

// One build attempt at the given count width; *out on success.
static scc_status build16(const scc_csr *g, const uint8_t *colors, int k, const scc16_build_opts &o, int bits,
                          bool validate, scc16_table **out)
{
    scc16_table *T = new scc16_table;
    T->k = k;
    T->rooting = o.rooting;
    T->n = g->n;
    T->nnz_g = g->nnz;
    T->chunk_terms = o.chunk_terms ? std::min(o.chunk_terms, MAX_CHUNK_TERMS) : DEFAULT_CHUNK_TERMS;
    T->stream = (hipStream_t)o.stream;
    T->mem.alloc = o.alloc;
    T->mem.stream = T->stream;
    T->count_bits = bits;
    T->info.n = g->n;
    T->info.k = k;
    T->info.rooting = o.rooting;
    T->info.count_bits = bits;
    scc_status s = SCC_OK;
    if (g->on_device) {
        T->row_ptr = g->row_ptr;
        T->col_idx = g->col_idx;
        T->colors = colors;
    } else {
        const int64_t n = g->n, nnz = g->nnz;
        int64_t *rp = (int64_t *)T->hold((size_t)(n + 1) * 8);
        int32_t *ci = (int32_t *)T->hold((size_t)std::max<int64_t>(nnz, 1) * 4);
        uint8_t *cl = (uint8_t *)T->hold((size_t)std::max<int64_t>(n, 1));
        if (!rp || !ci || !cl) s = set_error(SCC_ENOMEM, "graph copy");
        hipError_t e = hipSuccess;
        if (!s) e = hipMemcpyAsync(rp, g->row_ptr, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, T->stream);
        if (!s && e == hipSuccess && nnz > 0)
            e = hipMemcpyAsync(ci, g->col_idx, (size_t)nnz * 4, hipMemcpyHostToDevice, T->stream);
        if (!s && e == hipSuccess && n > 0) e = hipMemcpyAsync(cl, colors, (size_t)n, hipMemcpyHostToDevice, T->stream);
        if (!s && e == hipSuccess) e = hipStreamSynchronize(T->stream);
        if (!s && e != hipSuccess) s = set_error(SCC_EDEVICE, "graph copy: %s", hipGetErrorString(e));
        T->row_ptr = rp;
        T->col_idx = ci;
        T->colors = cl;
    }
    if (!s && validate) s = validate_csr(T->n, T->nnz_g, T->row_ptr, T->col_idx, T->colors, k, T->stream, T->mem);
    if (!s) s = bits == 256 ? build_all<U256>(T) : build_all<u128>(T);
    if (s) {
        delete T;
        return s;
    }
    int64_t bytes = 0;
    for (int h = 1; h <= k; h++) bytes += (T->n + 1) * 8 + T->X[h].nnz * (8 + bits / 8);
    T->info.bytes = bytes;
    for (int i = 0; i < 4; i++) T->info.t[i] = T->t[i];
    *out = T;
    return SCC_OK;
}

extern "C" scc_status scc16_build_table(const scc_csr *g, const uint8_t *colors, int k, const scc16_build_opts *opt,
                                        scc16_table **out)
{
    if (!out) return set_error(SCC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g || (g->n > 0 && !colors)) return set_error(SCC_EINVAL, "graph or colours NULL");
    if (k < 2 || k > K16) return set_error(SCC_EINVAL, "k = %d not in [2, 16]", k);
    if (g->n < 0 || g->n >= ((int64_t)1 << 31)) return set_error(SCC_EINVAL, "n out of range");
    if (g->nnz < 0 || g->nnz >= ((int64_t)1 << 40) || !g->row_ptr || (g->nnz > 0 && !g->col_idx))
        return set_error(SCC_EINVAL, "bad CSR pointers or size");
    scc16_build_opts o{};
    if (opt) o = *opt;
    if (o.rooting != SCC_ROOT_ZERO && o.rooting != SCC_ROOT_ALL)
        return set_error(SCC_EINVAL, "rooting must be SCC_ROOT_ZERO or SCC_ROOT_ALL");
    if (o.chunk_terms < 0) return set_error(SCC_EINVAL, "chunk_terms < 0");
    if (o.max_bits != 0 && o.max_bits != 128 && o.max_bits != 256)
        return set_error(SCC_EINVAL, "max_bits must be 0, 128 or 256");
    // 0: 128-bit counts, and the whole build again with 256-bit counts if a count
    // needs more than 128 bits
    scc_status s = build16(g, colors, k, o, o.max_bits == 256 ? 256 : 128, !o.no_validate, out);
    if (s == SCC_EOVERFLOW && o.max_bits == 0) s = build16(g, colors, k, o, 256, false, out);
    return s;
}

extern "C" void scc16_table_destroy(scc16_table *t) { delete t; }

extern "C" scc_status scc16_table_info_get(const scc16_table *t, scc16_table_info *out)
{
    if (!t || !out) return set_error(SCC_EINVAL, "NULL argument");
    *out = t->info;
    return SCC_OK;
}

extern "C" scc_status scc16_export_level(const scc16_table *t, int h, int64_t *nnz_out, int64_t *off, uint64_t *key,
                                         uint64_t *words, int nwords, void *stream)
{
    if (!t || !nnz_out) return set_error(SCC_EINVAL, "NULL argument");
    if (h < 1 || h > t->k) return set_error(SCC_EINVAL, "h = %d not in [1, %d]", h, t->k);
    const Lev16 &L = t->X[h];
    *nnz_out = L.nnz;
    if (!off) return SCC_OK;
    if (nwords != 2 && nwords != 4) return set_error(SCC_EINVAL, "nwords must be 2 or 4");
    if (nwords * 64 < t->count_bits)
        return set_error(SCC_EINVAL, "the table's counts are %d-bit: ask for 4 words", t->count_bits);
    if (L.nnz > 0 && (!key || !words)) return set_error(SCC_EINVAL, "NULL output array");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(off, L.off, (size_t)(t->n + 1) * 8, hipMemcpyDeviceToDevice, s));
    if (L.nnz > 0) {
        HIP_TRY(hipMemcpyAsync(key, L.key, (size_t)L.nnz * 8, hipMemcpyDeviceToDevice, s));
        if (t->count_bits == 256)
            hipLaunchKernelGGL((k16_words<U256>), dim3(blocks_for(L.nnz, 256)), dim3(256), 0, s, (const U256 *)L.cnt,
                               L.nnz, words, nwords);
        else
            hipLaunchKernelGGL((k16_words<u128>), dim3(blocks_for(L.nnz, 256)), dim3(256), 0, s, (const u128 *)L.cnt,
                               L.nnz, words, nwords);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(s));
    return SCC_OK;
}
