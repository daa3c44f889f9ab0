// The sampling phase on the GPU (Sec. 2.2) and the table's database queries
// occ(v), occ(T_C, v) (Sec. 3), plus export of stored records.
//
// One wave draws one sample. Every draw is a scan over a short list in a fixed
// order (vertices, record entries, colour sets, neighbours): the wave loads 64
// items, forms their inclusive running sum with shuffles, and the first lane
// whose running sum exceeds the drawn integer wins.
#include <cstring>

#include "sampler.hpp"

namespace {



__device__ inline int key_level(const DevLut &L, uint32_t key)
{
    int h = 1;
    while (h < L.k && (int)key >= L.off[h + 1]) h++;
    return h;
}

// first lane (in order) whose inclusive running sum exceeds `target`; -1 if none
__device__ inline int first_exceeding(u128 incl, u128 target)
{
    uint64_t bal = __ballot(incl > target);
    return bal ? __ffsll((long long)bal) - 1 : -1;
}

// First index j in [0, len) with val(j) > target, for a non-decreasing val whose
// last element exceeds target; -1 if it does not. While the range is large
// every lane probes one point (64-way split: the probes of the first rounds are
// shared by all samples and stay in cache); below 4096 entries only 8 lanes
// probe (8-way split), which keeps the per-search traffic to a few cache lines.
template <typename F>
__device__ inline int64_t wave_search(int64_t len, u128 target, F val)
{
    const int lane = lane_id();
    int64_t lo = 0;
    while (len > WAVE) {
        const int ways = len > 4096 ? WAVE : 8;
        const int64_t step = (len + ways - 1) / ways;
        const int64_t last = lo + len - 1;
        bool p = false;
        if (lane < ways) {
            int64_t idx = lo + (int64_t)(lane + 1) * step - 1;
            if (idx > last) idx = last;
            p = val(idx) > target;
        }
        const uint64_t bal = __ballot(p);
        if (!bal) return -1;                                 // target not below the last value
        const int f = __ffsll((long long)bal) - 1;
        const int64_t nlo = lo + (int64_t)f * step;
        const int64_t nhi = min(last, lo + (int64_t)(f + 1) * step - 1);
        lo = nlo;
        len = nhi - nlo + 1;
    }
    const bool p = lane < len && val(lo + lane) > target;
    const uint64_t bal = __ballot(p);
    if (!bal) return -1;
    return lo + (__ffsll((long long)bal) - 1);
}

// The draws of one sample, computed together: lane l holds the Philox block of
// (draw l % 16, attempt l / 16), so a draw reads its first four attempts from
// four lanes; later attempts (probability below 1/16) are computed one by one.
// The values are those of draw_below, bit for bit.
struct DrawCache {
    uint64_t lo, hi;
};

__device__ inline DrawCache draw_cache(uint64_t seed, uint64_t stream, uint64_t idx)
{
    const uint32_t lane = (uint32_t)lane_id();
    uint64_t c[4] = {idx, ((uint64_t)(lane % 16) << 32) | (lane / 16), 0, 0};
    philox4x64_10(c, seed, stream);
    return DrawCache{c[0], c[1]};
}


// value of lane src (src uniform), as a scalar
__device__ inline uint32_t readlane32(uint32_t x, int src) { return (uint32_t)__builtin_amdgcn_readlane((int)x, src); }
__device__ inline u128 readlane128(u128 x, int src) { return mk128(readlane64(lo64(x), src), readlane64(hi64(x), src)); }

__device__ inline u128 draw_cached(const DrawCache &D, u128 N, uint64_t seed, uint64_t stream, uint64_t idx,
                                   uint32_t draw)
{
    if (N <= 1) return 0;
    if (draw >= 16) return draw_below(N, seed, stream, idx, draw);
    const int bits = bitlen128(N - 1);
    const u128 mask = bits >= 128 ? ~(u128)0 : (((u128)1 << bits) - 1);
    for (uint32_t att = 0; att < 4; att++) {
        const int src = (int)(draw + 16 * att);
        const u128 x = mk128(readlane64(D.lo, src), readlane64(D.hi, src)) & mask;
        if (x < N) return x;
    }
    for (uint32_t att = 4; att < 4096u; att++) {
        uint64_t c[4] = {idx, ((uint64_t)draw << 32) | att, 0, 0};
        philox4x64_10(c, seed, stream);
        const u128 x = mk128(c[0], c[1]) & mask;
        if (x < N) return x;
    }
    return N - 1;
}

// count of (T, C) with the given key at x (level h >= 1), x of colour cx
__device__ inline u128 own_count_c(const SampleArgs &A, int h, int64_t x, int cx, uint32_t key)
{
    if (h == 1) return (key == (uint32_t)cx) ? 1 : 0;   // key of ({.}, {c}) is c
    const int li = A.key_xidx[(size_t)cx * A.nkeys + key];
    if (li < 0) return 0;
    // dense position li: its bitmap word, then the popcount of the words before
    // it gives the entry; the locator goes out with the word
    const LevelView &L = A.lev[h];
    const uint64_t *bw = L.bm + (size_t)x * L.BW;
    const int w = li >> 6;
    const uint64_t l = L.loc[x];
    const uint64_t word = bw[w];
    // an empty record has no bit set: testing its locator as well keeps the
    // locator's load beside the word's instead of after the test
    if (!((word >> (li & 63)) & 1ull) || !l) return 0;
    uint32_t pos = (uint32_t)__popcll(word & ((1ull << (li & 63)) - 1ull));
    int q = 0;
    for (; q + 1 < w; q += 2) {   // two words per load
        const uint64_t a = bw[q], b = bw[q + 1];
        pos += (uint32_t)(__popcll(a) + __popcll(b));
    }
    if (q < w) pos += (uint32_t)__popcll(bw[q]);
    Rec r;
    r.len = LOC_LEN(l);
    r.wide = LOC_WIDE(l) != 0;
    r.vlc = L.vlc != 0;
    r.kw = key_words(r.len);
    r.p = L.pool + LOC_OFF(l);
    return r.cnt(pos);
}
__device__ inline u128 own_count(const SampleArgs &A, int h, int64_t x, uint32_t key)
{
    return own_count_c(A, h, x, A.g.colors[x], key);
}
// colour of the head of edge e (u = col_idx[e])
__device__ inline int edge_colour(const SampleArgs &A, int64_t e, int32_t u)
{
    return A.ecol ? A.ecol[e] : A.g.colors[u];
}

// LDS of one wave's sample: the vertices found so far with their parents, and
// the stack of pending decompositions (key, position of its root, count)
struct SampleLds {
    int32_t sv[SCC_KMAX];
    int8_t par[SCC_KMAX];
    uint32_t st_key[2 * SCC_KMAX];
    int st_pos[2 * SCC_KMAX];
    u128 st_cnt[2 * SCC_KMAX];
};

// An uncoloured k-star (round skipping, Sec. 3.3): the centre v by its running
// sum of binom(d_v, k-1) (draw 0), then the i-th leaf at position r uniform
// below d_v - i (draw 1 + i) among the neighbours not taken yet, where a taken
// position is refilled by the last remaining one. Every lane makes the same
// draws; lane q < i holds the q-th refilled position and its current value.
__device__ inline int sample_star(const SampleArgs &A, int64_t r)
{
    const int lane = lane_id();
    const int k = A.k;
    const uint64_t idx = A.first + (uint64_t)r;
    const DrawCache D = draw_cache(A.seed, A.stream, idx);
    const u128 X = draw_cached(D, A.total, A.seed, A.stream, idx, 0);
    const int64_t v = wave_search(A.g.n, X, [&](int64_t i) { return A.pre[i]; });
    if (v < 0) return 4;
    const int64_t ra = A.g.row_ptr[v], d = A.g.row_ptr[v + 1] - ra;
    if (d < k - 1) return 4;
    int64_t mpos = -1, mval = 0;     // this lane's refilled position
    int nm = 0;
    int32_t leaf = (int32_t)v;
    for (int i = 0; i < k - 1; i++) {
        const int64_t rr = (int64_t)draw_cached(D, (u128)(d - i), A.seed, A.stream, idx, 1 + i);
        const int64_t last = d - 1 - i;
        const uint64_t hit = __ballot(lane < nm && mpos == rr);
        const uint64_t hitl = __ballot(lane < nm && mpos == last);
        // (the hit lanes are the wave's common choice: their values read as scalars)
        const int64_t got = hit ? (int64_t)readlane64((uint64_t)mval, __ffsll((long long)hit) - 1) : rr;
        const int64_t lastval = hitl ? (int64_t)readlane64((uint64_t)mval, __ffsll((long long)hitl) - 1) : last;
        if (lane == 1 + i) leaf = A.g.col_idx[ra + got];
        const int q = hit ? __ffsll((long long)hit) - 1 : nm;
        if (lane == q) { mpos = rr; mval = lastval; }
        if (!hit) nm++;
    }
    if (lane < k) {
        A.verts[(size_t)r * k + lane] = leaf;
        A.par[(size_t)r * k + lane] = lane == 0 ? -1 : 0;
    }
    return 0;
}

// Sample number r of A's stream (random index A.first + r) into row r of
// A.verts / A.par, by the whole wave. Returns 0, or an error bit (1: the root
// entry draw fell off the record, 2: a decomposition draw failed, 4: the root
// vertex (or shape) draw fell off its running sums); none is expected for a
// consistent table.
__device__ inline int sample_one(const SampleArgs &A, int64_t r, SampleLds &W)
{
    if (A.mode == 2) return sample_star(A, r);
    int32_t *sv = W.sv;
    int8_t *sp_par = W.par;
    uint32_t *st_key = W.st_key;
    int *st_pos = W.st_pos;
    u128 *st_cnt = W.st_cnt;
    const DevLut &L = *A.L;
    const int lane = lane_id();
    const int k = A.k;
    const uint64_t idx = A.first + (uint64_t)r;
    const DrawCache D = draw_cache(A.seed, A.stream, idx);
    int shape = A.shape;
    const u128 *pre = A.pre;
    u128 total = A.total;
    uint32_t doff = 0;   // draw numbers start here
    if (A.mode == 1) {
        // shape first: j with running sum of t_j (ascending) exceeding X0, then
        // shape j's draws numbered from 1
        const u128 X0 = draw_cached(D, A.total, A.seed, A.stream, idx, 0);
        const u128 incl = wave_incl_scan128(lane < L.num_unr ? A.stj[lane] : (u128)0);
        const int j = first_exceeding(incl, X0);
        if (j < 0) return 4;
        shape = j;
        pre = A.spre[j];
        total = pre[A.g.n - 1];
        doff = 1;
    }
    // (1) root: first vertex whose running sum exceeds X, then the entry of its record
    const u128 X = draw_cached(D, total, A.seed, A.stream, idx, doff);
    const int64_t v = wave_search(A.g.n, X, [&](int64_t i) { return pre[i]; });
    if (v < 0) return 4;
    const u128 res = X - (v > 0 ? pre[v - 1] : (u128)0);
    const Rec rk = rec_of(A.lev[k], v);
    const uint32_t lenk = rk.len;
    u128 run = 0;
    uint32_t rkey = 0xffffffffu;
    u128 rcnt = 0;
    for (uint32_t b0 = 0; b0 < lenk; b0 += WAVE) {
        const uint32_t e = b0 + lane;
        u128 c = 0;
        uint32_t key = 0;
        if (e < lenk) {
            key = rk.key(e);
            const int t = (int)(key - L.off[k]) / L.bk[k];
            if (shape < 0 || L.unr_of[t] == shape) c = rk.cnt(e);
        }
        const u128 incl = run + wave_incl_scan128(c);
        const int w = first_exceeding(incl, res);
        if (w >= 0) {
            rkey = readlane32(key, w);
            rcnt = readlane128(c, w);
            break;
        }
        run = readlane128(incl, WAVE - 1);
    }
    if (rkey == 0xffffffffu) return 1;
    if (lane == 0) {
        sv[0] = (int32_t)v; sp_par[0] = -1;
        st_key[0] = rkey; st_pos[0] = 0; st_cnt[0] = rcnt;
    }
    __syncthreads();
    int nv = 1, sp = 1, dec = 0;
    bool fail = false;
    // (2) decompose, LIFO: (T', C \ C'', x) is processed before (T'', C'', u)
    while (sp > 0 && !fail) {
        sp--;
        // every lane reads the same LDS words: made scalar, so that the per-level
        // arrays below are addressed from scalar registers
        const uint32_t key = (uint32_t)__builtin_amdgcn_readfirstlane((int)st_key[sp]);
        const int pos = __builtin_amdgcn_readfirstlane(st_pos[sp]);
        const u128 cT = mk128(readfirst64(lo64(st_cnt[sp])), readfirst64(hi64(st_cnt[sp])));
        __syncthreads();
        const int h = key_level(L, key);
        if (h == 1) continue;
        const int rel = (int)key - L.off[h];
        const int t = rel / L.bk[h];
        const uint32_t C = L.mask_k[h][rel - t * L.bk[h]];
        const int64_t x = __builtin_amdgcn_readfirstlane(sv[pos]);
        const int cx = A.g.colors[x];
        const int hp = L.dec_hp[h][t], hpp = h - hp, a = L.dec_a[h][t], b = L.dec_b[h][t];
        const int beta = L.dec_beta[h][t];
        const u128 Y = draw_cached(D, (u128)beta * cT, A.seed, A.stream, idx, doff + 1 + 2 * dec);
        // stage 1: C'' among the |T''|-subsets of C \ {c_x}, ascending bitmask
        const uint32_t R = C & ~(1u << cx);
        int ncand = 1;
        for (int i = 1; i <= hpp; i++) ncand = ncand * (h - 1 - hpp + i) / i;
        u128 w = 0, xprime = 0, sval = 0;
        uint32_t cpp = 0;
        int sidx = 0;
        if (lane < ncand) {
            // deposit the lane-th hpp-subset of the low h-1 positions onto R's bits
            uint32_t pm = L.mask_s[hpp][lane], dep = 0, rr = R;
            for (int q = 0; rr; q++) {
                const uint32_t bit = rr & (~rr + 1u);
                if (pm >> q & 1u) dep |= bit;
                rr &= rr - 1u;
            }
            cpp = dep;
            const uint32_t kprime = L.off[hp] + a * L.bk[hp] + L.colex_k[C ^ cpp];
            xprime = own_count(A, hp, x, kprime);
            const int ws = L.WS[hpp];
            sidx = b * L.bk1[hpp] + L.colex_s[compress_out(cpp, cx)];
            const uint64_t slo = A.Slo[hpp][(size_t)x * ws + sidx];
            const uint64_t shi =
                hi64(A.M[hpp][x]) ? A.Shi[hpp][(A.Shrow[hpp] ? (size_t)A.Shrow[hpp][x] : (size_t)x) * ws + sidx] : 0;
            sval = mk128(slo, shi);
            w = xprime * sval;
        }
        const u128 incl1 = wave_incl_scan128(w);
        const int w1 = first_exceeding(incl1, Y);
        if (w1 < 0) { fail = true; break; }
        // the chosen candidate's values, read from its lane as scalars
        const uint32_t Cpp = readlane32(cpp, w1);
        const int Sidx = (int)readlane32((uint32_t)sidx, w1);
        const u128 Xp = readlane128(xprime, w1);
        const u128 Sv = readlane128(sval, w1);
        // stage 2: neighbour u of x with weight c(T''_{C''}, u), CSR order
        const u128 Z = draw_cached(D, Sv, A.seed, A.stream, idx, doff + 2 + 2 * dec);
        const uint32_t kpp = L.off[hpp] + b * L.bk[hpp] + L.colex_k[Cpp];
        const int64_t ra = A.g.row_ptr[x], rb = A.g.row_ptr[x + 1];
        int64_t u = -1;
        u128 wu = 0;
        const int hub = A.hub_index ? A.hub_index[x] : -1;
        if (hub >= 0) {
            // running sums over x's neighbours at the end of every block of HUB_BLOCK
            // neighbours, precomputed per (hub, level, entry): search the block, then
            // scan its neighbours from the running sum before it
            const int64_t d = rb - ra, nb = (d + HUB_BLOCK - 1) / HUB_BLOCK;
            const int64_t base = A.hub_poff[(size_t)hub * (SCC_KMAX + 1) + hpp];
            const uint64_t *plo = A.hub_pre + base + (size_t)Sidx * nb;
            const bool pw = hi64(A.M[hpp][x]) != 0;
            const uint64_t *phi = A.hub_pre + base + (size_t)L.WS[hpp] * nb + (size_t)Sidx * nb;
            auto P = [&](int64_t j) { return mk128(plo[j], pw ? phi[j] : 0); };
            const int64_t b = wave_search(nb, Z, P);
            if (b >= 0) {
                const int64_t e = ra + b * HUB_BLOCK + lane;
                u128 c = 0;
                int32_t uu = -1;
                if (e < rb) {
                    uu = A.g.col_idx[e];
                    c = own_count_c(A, hpp, uu, edge_colour(A, e, uu), kpp);
                }
                const u128 incl = (b > 0 ? P(b - 1) : (u128)0) + wave_incl_scan128(c);
                const int w2 = first_exceeding(incl, Z);
                if (w2 >= 0) {
                    u = (int32_t)readlane32((uint32_t)uu, w2);
                    wu = readlane128(c, w2);
                }
            }
        } else {
            // CSR order, 2 x 64 neighbours per round: every lane issues the loads of
            // its 2 neighbours (and their colours, stored per edge) before using any,
            // then the 2 groups are scanned in order
            u128 run2 = 0;
            bool found = false;
            for (int64_t base = ra; base < rb && !found; base += 2 * WAVE) {
                int32_t uu[2];
                int cu[2];
                u128 c[2];
#pragma unroll
                for (int g4 = 0; g4 < 2; g4++) {
                    const int64_t e = base + g4 * WAVE + lane;
                    uu[g4] = e < rb ? A.g.col_idx[e] : -1;
                    cu[g4] = e < rb && A.ecol ? A.ecol[e] : 0;
                }
#pragma unroll
                for (int g4 = 0; g4 < 2; g4++)
                    c[g4] = uu[g4] >= 0 ? own_count_c(A, hpp, uu[g4], A.ecol ? cu[g4] : A.g.colors[uu[g4]], kpp)
                                        : (u128)0;
#pragma unroll
                for (int g4 = 0; g4 < 2; g4++) {
                    if (found) break;
                    const u128 incl = run2 + wave_incl_scan128(c[g4]);
                    const int w2 = first_exceeding(incl, Z);
                    if (w2 >= 0) {
                        u = (int32_t)readlane32((uint32_t)uu[g4], w2);
                        wu = readlane128(c[g4], w2);
                        found = true;
                    } else {
                        run2 = readlane128(incl, WAVE - 1);
                    }
                }
            }
        }
        if (u < 0) { fail = true; break; }
        if (lane == 0) {
            sv[nv] = (int32_t)u;
            sp_par[nv] = (int8_t)pos;
            st_key[sp] = kpp; st_pos[sp] = nv; st_cnt[sp] = wu;
            st_key[sp + 1] = L.off[hp] + a * L.bk[hp] + L.colex_k[C ^ Cpp];
            st_pos[sp + 1] = pos; st_cnt[sp + 1] = Xp;
        }
        __syncthreads();
        nv++;
        sp += 2;
        dec++;
    }
    if (fail || nv != k) return 2;
    if (lane < k) {
        A.verts[(size_t)r * k + lane] = sv[lane];
        A.par[(size_t)r * k + lane] = sp_par[lane];
    }
    return 0;
}

// the draws are latency-bound: eight waves per SIMD (with the chosen lanes'
// values kept in scalar registers the sampler needs at most 64 registers)
// measured 12 % faster than seven and than six
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(8, 8))) k_sample(SampleArgs A)
{
    __shared__ SampleLds W;
    for (int64_t s = blockIdx.x; s < A.nsamp; s += gridDim.x) {
        const int e = sample_one(A, s, W);
        if (e && lane_id() == 0) atomicOr(A.err, e);
        __syncthreads();
    }
}

// A serving step: rows of many requests (each with its own table, shape and
// random stream), flattened; row s belongs to the first chunk whose running end
// exceeds s. The grid strides over the rows.
// (eight waves per SIMD, as the plain sampler)
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(8, 8))) k_serve_sample(const SampleArgs *args, const ServeChunk *ch,
                                                      const int64_t *cend, int nch, int64_t total, int *err)
{
    __shared__ SampleLds W;
    for (int64_t s = blockIdx.x; s < total; s += gridDim.x) {
        int lo = 0, hi = nch - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cend[mid] > s) hi = mid; else lo = mid + 1;
        }
        const ServeChunk C = ch[lo];
        const int64_t r = C.off + (s - (cend[lo] - C.count));
        const SampleArgs &A = *(const SampleArgs *)((const __attribute__((address_space(4))) SampleArgs *)args + C.arg);
        const int e = sample_one(A, r, W);
        if (e && lane_id() == 0) atomicOr(err, e);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Per-hub running sums for the neighbour draw. For hub x, level h'' and
// neighbour-sum entry s (the (T'', C'') seen from x), row s of the (x, h'')
// block holds sum_{i <= j} c(T''_{C''}, u_i) over x's neighbours u_0, u_1, ...
// ---------------------------------------------------------------------------
struct HubPreArgs {
    GraphView g;
    const DevLut *L;
    int k, nkeys, zero;
    LevelView lev[SCC_KMAX + 1];
    const u128 *M[SCC_KMAX + 1];
    const int16_t *key_sidx;
    const int32_t *hubs;
    const int64_t *hub_rows;     // [2 * nhub]
    const int64_t *poff;         // [nhub * (k+1)]
    uint64_t *pre;
    const int32_t *chunk_hub;    // hub number of each chunk
    const int64_t *chunk_e;      // first edge of each chunk
    const int32_t *hub_first_chunk;
    const int16_t *key_xidx;
    u128 *part;                  // chunk totals, part_stride entries per chunk
    int part_stride;
    int chunk;
};

// inclusive scan over a 256-thread workgroup (4 waves)
__device__ inline u128 block256_incl_scan(u128 x, u128 *ws)
{
    x = wave_incl_scan128(x);
    if (lane_id() == WAVE - 1) ws[threadIdx.x / WAVE] = x;
    __syncthreads();
    u128 before = 0;
    for (int w = 0; w < (int)(threadIdx.x / WAVE); w++) before += ws[w];
    __syncthreads();
    return x + before;
}

// one neighbour's record location, read once and reused for every entry
struct NbrRec {
    const uint64_t *rec;    // count words (low), after the keys
    const uint64_t *bm;     // presence bitmap
    uint32_t len;
    bool wide;
    int cu;
};

__device__ inline NbrRec nbr_load(const HubPreArgs &A, int hpp, int32_t u)
{
    NbrRec r{nullptr, nullptr, 0, false, 0};
    if (u < 0) return r;
    r.cu = A.g.colors[u];
    if (hpp == 1) return r;
    const LevelView &L = A.lev[hpp];
    const Rec rr = rec_of(L, u);
    r.len = rr.len;
    r.wide = rr.wide;
    r.bm = L.bm + (size_t)u * L.BW;
    if (r.len) r.rec = rr.p + REC_HDR + rr.kw;
    return r;
}

__device__ inline u128 nbr_count(const HubPreArgs &A, int hpp, const NbrRec &r, uint32_t key)
{
    if (hpp == 1) return key == (uint32_t)r.cu ? 1 : 0;
    const int li = A.key_xidx[(size_t)r.cu * A.nkeys + key];
    if (li < 0 || !r.len) return 0;
    const uint64_t word = r.bm[li >> 6];
    if (!((word >> (li & 63)) & 1ull)) return 0;
    uint32_t pos = (uint32_t)__popcll(word & ((1ull << (li & 63)) - 1ull));
    for (int q = 0; q < (li >> 6); q++) pos += (uint32_t)__popcll(r.bm[q]);
    return mk128(r.rec[pos], r.wide ? r.rec[r.len + pos] : 0);
}

// pass 1: per (chunk of HUBPRE_CHUNK neighbours of a hub, level): the values of
// every entry for every neighbour of the chunk, scanned within the chunk
// (writes are coalesced along the neighbour axis); chunk totals go to `part`
__global__ void __launch_bounds__(256) k_hubpre_chunk(HubPreArgs A)
{
    __shared__ uint32_t skey[192];
    __shared__ u128 ws[256 / WAVE];
    __shared__ u128 carry;
    const int c = blockIdx.x;
    const int q = A.chunk_hub[c];
    const int hpp = blockIdx.y + 1;
    const int64_t x = A.hubs[q];
    const int cx = A.g.colors[x];
    if (A.zero && hpp == A.k - 1 && cx != 0) return;   // no block: x is never a root there
    if (!A.M[hpp]) return;                              // no block: sums not built
    const DevLut &L = *A.L;
    const int WS = L.WS[hpp];
    const int64_t ra = A.hub_rows[2 * q], rb = A.hub_rows[2 * q + 1], d = rb - ra;
    const int64_t e0 = A.chunk_e[c], e1 = min(rb, e0 + (int64_t)A.chunk);
    const bool pw = hi64(A.M[hpp][x]) != 0;
    const int64_t nb = (d + HUB_BLOCK - 1) / HUB_BLOCK;
    uint64_t *plo = A.pre + A.poff[(size_t)q * (SCC_KMAX + 1) + hpp];
    uint64_t *phi = plo + (size_t)WS * nb;
    for (int t = threadIdx.x; t < WS; t += blockDim.x) {
        const int rank = t / L.bk1[hpp], dc = t - rank * L.bk1[hpp];
        const uint32_t C = expand_in(L.mask_s[hpp][dc], cx);
        skey[t] = (uint32_t)(L.off[hpp] + rank * L.bk[hpp] + L.colex_k[C]);
    }
    int32_t u[4];
    NbrRec nr[4];
    for (int r = 0; r < 4; r++) {
        const int64_t e = e0 + r * 256 + threadIdx.x;
        u[r] = e < e1 ? A.g.col_idx[e] : -1;
        nr[r] = nbr_load(A, hpp, u[r]);
    }
    __syncthreads();
    for (int sidx = 0; sidx < WS; sidx++) {
        const uint32_t key = skey[sidx];
        u128 run = 0;
        for (int r = 0; r < 4 && e0 + r * 256 < e1; r++) {
            const u128 val = u[r] >= 0 ? nbr_count(A, hpp, nr[r], key) : (u128)0;
            const u128 inc = block256_incl_scan(val, ws) + run;
            const int64_t j = e0 + r * 256 + threadIdx.x - ra;
            if (u[r] >= 0 && ((j % HUB_BLOCK) == HUB_BLOCK - 1 || j == d - 1)) {   // end of a block
                plo[(size_t)sidx * nb + j / HUB_BLOCK] = lo64(inc);
                if (pw) phi[(size_t)sidx * nb + j / HUB_BLOCK] = hi64(inc);
            }
            if (threadIdx.x == blockDim.x - 1) carry = inc;
            __syncthreads();
            run = carry;
            __syncthreads();
        }
        if (threadIdx.x == 0) A.part[(size_t)c * A.part_stride + L.soff[hpp] + sidx] = run;
    }
}

// pass 2: add the totals of a hub's earlier chunks to every later chunk
__global__ void __launch_bounds__(256) k_hubpre_fix(HubPreArgs A)
{
    __shared__ u128 add[192];
    const int c = blockIdx.x;
    const int q = A.chunk_hub[c];
    const int first = A.hub_first_chunk[q];
    if (c == first) return;
    const int hpp = blockIdx.y + 1;
    const int64_t x = A.hubs[q];
    if (A.zero && hpp == A.k - 1 && A.g.colors[x] != 0) return;
    if (!A.M[hpp]) return;
    const DevLut &L = *A.L;
    const int WS = L.WS[hpp];
    const int64_t ra = A.hub_rows[2 * q], rb = A.hub_rows[2 * q + 1], d = rb - ra;
    const int64_t e0 = A.chunk_e[c], e1 = min(rb, e0 + (int64_t)A.chunk);
    const bool pw = hi64(A.M[hpp][x]) != 0;
    const int64_t nb = (d + HUB_BLOCK - 1) / HUB_BLOCK;
    uint64_t *plo = A.pre + A.poff[(size_t)q * (SCC_KMAX + 1) + hpp];
    uint64_t *phi = plo + (size_t)WS * nb;
    for (int t = threadIdx.x; t < WS; t += blockDim.x) {
        u128 o = 0;
        for (int cc = first; cc < c; cc++) o += A.part[(size_t)cc * A.part_stride + L.soff[hpp] + t];
        add[t] = o;
    }
    __syncthreads();
    // the chunk's blocks (chunks start on block boundaries)
    const int64_t b0 = (e0 - ra) / HUB_BLOCK, b1 = (e1 - ra + HUB_BLOCK - 1) / HUB_BLOCK, len = b1 - b0;
    for (int64_t i = threadIdx.x; i < (int64_t)WS * len; i += blockDim.x) {
        const int sidx = (int)(i / len);
        const int64_t j = b0 + (i - (int64_t)sidx * len);
        const u128 o = add[sidx];
        const u128 cur = mk128(plo[(size_t)sidx * nb + j], pw ? phi[(size_t)sidx * nb + j] : 0);
        const u128 nv = cur + o;
        plo[(size_t)sidx * nb + j] = lo64(nv);
        if (pw) phi[(size_t)sidx * nb + j] = hi64(nv);
    }
}

__global__ void k_hub_index(const int32_t *hubs, int nhub, int32_t *index)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nhub) index[hubs[i]] = i;
}

__global__ void k_occ(GraphView g, const DevLut *Lp, LevelView lev_h, int h, int64_t v, int32_t key,
                      const u128 *eta, u128 *out)
{
    if (threadIdx.x != 0) return;
    if (key < 0) { *out = eta[v]; return; }
    if (h == 1) { *out = ((uint32_t)key == g.colors[v]) ? 1 : 0; return; }
    *out = record_lookup(lev_h, v, (uint32_t)key);
}

__global__ void k_len(int64_t n, const uint64_t *loc, int h1, const uint8_t *colors, uint64_t *len)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    len[v] = h1 ? 1 : LOC_LEN(loc[v]);
}

__global__ void __launch_bounds__(WAVE) k_export(int64_t n, LevelView Lv, int h1, const uint8_t *colors,
                                                 const uint64_t *incl, int64_t *off, uint16_t *key,
                                                 uint64_t *lo, uint64_t *hi)
{
    const int64_t v = blockIdx.x;
    const int lane = threadIdx.x;
    const uint64_t end = incl[v];
    if (h1) {
        if (lane == 0) {
            off[v] = (int64_t)end - 1;
            if (v == n - 1) off[n] = (int64_t)end;
            key[end - 1] = colors[v];
            lo[end - 1] = 1;
            hi[end - 1] = 0;
        }
        return;
    }
    const Rec r = rec_of(Lv, v);
    const uint64_t start = end - r.len;
    if (lane == 0) {
        off[v] = (int64_t)start;
        if (v == n - 1) off[n] = (int64_t)end;
    }
    for (uint32_t e = lane; e < r.len; e += WAVE) {
        key[start + e] = (uint16_t)r.key(e);
        lo[start + e] = r.lo(e);
        hi[start + e] = r.hi(e);
    }
}

LevelView lview(const TableLevel &l) { return LevelView{l.pool, l.loc, l.bm, l.BW, l.vlc ? 1 : 0}; }

}  // namespace

__global__ void k_hub_info(const int32_t *hubs, int nhub, int k, const uint8_t *colors, HubPreArgs A, uint8_t *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nhub) return;
    const int64_t x = hubs[i];
    out[(size_t)i * (SCC_KMAX + 2)] = colors[x];
    for (int h = 1; h < k; h++) out[(size_t)i * (SCC_KMAX + 2) + h] = A.M[h] && hi64(A.M[h][x]) ? 1 : 0;
}

// colour of every edge's head, in CSR order
__global__ void k_edge_colours(const int32_t *col_idx, const uint8_t *colors, int64_t nnz, uint8_t *ecol)
{
    const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
#pragma unroll
    for (int j = 0; j < 4; j++)
        if (e0 + j < nnz) ecol[e0 + j] = colors[col_idx[e0 + j]];
}

// The per-edge colours of the neighbour draw (nnz bytes, built once per table).
static scc_status ensure_edge_colours(scc_table *T)
{
    std::lock_guard<std::mutex> g(T->hub_mu);
    if (T->ecol || T->nnz_g == 0) return SCC_OK;
    uint8_t *ec = (uint8_t *)T->alloc((size_t)T->nnz_g + 8);
    if (!ec) return set_error(SCC_ENOMEM, "edge colours (%lld bytes)", (long long)T->nnz_g);
    const int64_t nt = (T->nnz_g + 3) / 4;
    hipLaunchKernelGGL(k_edge_colours, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, T->stream, T->col_idx,
                       T->colors, T->nnz_g, ec);
    HIP_TRY(hipStreamSynchronize(T->stream));
    HIP_TRY(hipGetLastError());
    T->ecol = ec;
    return SCC_OK;
}

// Builds the per-hub running sums used by the sampler's neighbour draw. Hubs
// are taken by decreasing degree while the tables fit in `budget` bytes.
static scc_status ensure_hub_prefix(scc_table *T)
{
    std::lock_guard<std::mutex> g(T->hub_mu);
    if (T->hubpre_ready) return SCC_OK;
    const int k = T->k;
    const int nh = (int)T->hub_host.size();
    hipStream_t st = T->stream;
    if (nh == 0 || k < 2) { T->hubpre_ready = true; return SCC_OK; }
    if (T->vlc) return set_error(SCC_EINVAL, "internal: hub running sums after the variable-length re-encoding");
    const DevLut &HL = T->hlut;
    HubPreArgs A{};
    A.g = GraphView{T->n, T->row_ptr, T->col_idx, T->colors};
    A.L = T->dlut; A.k = k; A.nkeys = HL.nkeys; A.zero = T->rooting == SCC_ROOT_ZERO;
    for (int h = 2; h <= k; h++) A.lev[h] = lview(T->lev[h]);
    for (int h = 1; h < k; h++) A.M[h] = T->S[h].M;
    A.key_sidx = T->key_sidx;
    std::vector<void *> tmp;
    auto get = [&](size_t b) { void *p = T->mem.get(b); if (p) tmp.push_back(p); return p; };
    struct Free { scc_table *T; std::vector<void *> *v; ~Free() { for (void *p : *v) T->mem.put(p); } } fr{T, &tmp};
    int32_t *dh = (int32_t *)get((size_t)nh * 4);
    uint8_t *dinfo = (uint8_t *)get((size_t)nh * (SCC_KMAX + 2));
    if (!dh || !dinfo) return set_error(SCC_ENOMEM, "hub info");
    HIP_TRY(hipMemcpyAsync(dh, T->hub_host.data(), (size_t)nh * 4, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_hub_info, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, st, dh, nh, k, T->colors, A, dinfo);
    std::vector<uint8_t> info((size_t)nh * (SCC_KMAX + 2));
    HIP_TRY(hipMemcpyAsync(info.data(), dinfo, info.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    // choose hubs by decreasing degree within the budget
    std::vector<int> order(nh);
    for (int i = 0; i < nh; i++) order[i] = i;
    auto deg = [&](int i) { return T->hub_rows_host[2 * i + 1] - T->hub_rows_host[2 * i]; };
    std::sort(order.begin(), order.end(), [&](int a, int b) { return deg(a) > deg(b); });
    const bool zero = T->rooting == SCC_ROOT_ZERO;
    auto block_words = [&](int i, int h) -> int64_t {
        if (zero && h == k - 1 && info[(size_t)i * (SCC_KMAX + 2)] != 0) return 0;   // never a root there
        if (!T->S[h].M) return 0;                                                      // sums not built
        const int64_t w = (int64_t)HL.WS[h] * ((deg(i) + HUB_BLOCK - 1) / HUB_BLOCK);
        return info[(size_t)i * (SCC_KMAX + 2) + h] ? 2 * w : w;
    };
    const int64_t budget_words = T->hub_prefix_budget / 8;
    std::vector<int> chosen;
    int64_t total = 0;
    for (int i : order) {
        int64_t w = 0;
        for (int h = 1; h < k; h++) w += block_words(i, h);
        if (total + w > budget_words) break;
        total += w;
        chosen.push_back(i);
    }
    std::sort(chosen.begin(), chosen.end());
    const int nc = (int)chosen.size();
    T->hub_count_pre = nc;
    if (nc == 0) { T->hubpre_ready = true; return SCC_OK; }
    std::vector<int32_t> hubs(nc);
    std::vector<int64_t> rows(2 * (size_t)nc), poff((size_t)nc * (SCC_KMAX + 1), 0);
    std::vector<int32_t> ch, first(nc);
    std::vector<int64_t> ce;
    int64_t at = 0;
    const int CH = 1024;
    for (int q = 0; q < nc; q++) {
        const int i = chosen[q];
        hubs[q] = T->hub_host[i];
        rows[2 * q] = T->hub_rows_host[2 * i];
        rows[2 * q + 1] = T->hub_rows_host[2 * i + 1];
        for (int h = 1; h < k; h++) { poff[(size_t)q * (SCC_KMAX + 1) + h] = at; at += block_words(i, h); }
        first[q] = (int32_t)ch.size();
        for (int64_t e = rows[2 * q]; e < rows[2 * q + 1]; e += CH) { ch.push_back(q); ce.push_back(e); }
    }
    T->hub_pre = (uint64_t *)T->alloc((size_t)at * 8 + 8);
    T->hub_poff = (int64_t *)T->alloc(poff.size() * 8);
    T->hub_index = (int32_t *)T->alloc((size_t)T->n * 4 + 4);
    int32_t *dhubs = (int32_t *)T->alloc((size_t)nc * 4);
    int64_t *drows = (int64_t *)get(rows.size() * 8);
    int32_t *dch = (int32_t *)get(ch.size() * 4);
    int64_t *dce = (int64_t *)get(ce.size() * 8);
    int32_t *dfirst = (int32_t *)get((size_t)nc * 4);
    const int pstride = HL.soff[k];
    u128 *dpart = (u128 *)get(ch.size() * (size_t)pstride * 16 + 16);
    if (!T->hub_pre || !T->hub_poff || !T->hub_index || !dhubs || !drows || !dch || !dce || !dfirst || !dpart)
        return set_error(SCC_ENOMEM, "hub running sums (%lld bytes)", (long long)at * 8);
    HIP_TRY(hipMemcpyAsync(dfirst, first.data(), (size_t)nc * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(T->hub_index, 0xff, (size_t)T->n * 4, st));
    HIP_TRY(hipMemcpyAsync(T->hub_poff, poff.data(), poff.size() * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dhubs, hubs.data(), (size_t)nc * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(drows, rows.data(), rows.size() * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dch, ch.data(), ch.size() * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dce, ce.data(), ce.size() * 8, hipMemcpyHostToDevice, st));
    A.hubs = dhubs; A.hub_rows = drows; A.poff = T->hub_poff; A.pre = T->hub_pre;
    A.chunk_hub = dch; A.chunk_e = dce; A.chunk = CH; A.hub_first_chunk = dfirst;
    A.key_xidx = T->key_xidx; A.part = dpart; A.part_stride = pstride;
    hipLaunchKernelGGL(k_hub_index, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, dhubs, nc, T->hub_index);
    hipLaunchKernelGGL(k_hubpre_chunk, dim3((unsigned)ch.size(), (unsigned)(k - 1)), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_hubpre_fix, dim3((unsigned)ch.size(), (unsigned)(k - 1)), dim3(256), 0, st, A);
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipGetLastError());
    T->hubpre_ready = true;
    return SCC_OK;
}

scc_status table_prefix(scc_table *T, int shape, const u128 **pre, u128 *total)
{
    if (shape < 0) {
        *pre = T->pre;
        *total = T->root_total;
        return SCC_OK;
    }
    std::lock_guard<std::mutex> g(T->mu);
    auto it = T->pre_shape.find(shape);
    if (it != T->pre_shape.end()) {
        *pre = it->second;
        *total = T->tot_shape[shape];
        return SCC_OK;
    }
    const int64_t n = T->n;
    u128 *eta = (u128 *)T->mem.get((size_t)n * 16 + 16);
    u128 *p = (u128 *)T->alloc((size_t)n * 16 + 16);
    if (!eta || !p) { T->mem.put(eta); return set_error(SCC_ENOMEM, "shape prefix"); }
    launch_eta_shape(T, shape, eta);
    scc_status s = scan_u128(T, eta, p, n);
    T->mem.put(eta);
    if (s) return s;
    u128 tot = 0;
    if (n) {
        HIP_TRY(hipMemcpyAsync(&tot, p + (n - 1), 16, hipMemcpyDeviceToHost, T->stream));
        HIP_TRY(hipStreamSynchronize(T->stream));
    }
    T->pre_shape[shape] = p;
    T->tot_shape[shape] = tot;
    *pre = p;
    *total = tot;
    return SCC_OK;
}

// Round skipping, shape -1: every non-star shape's root running sums and the
// device arrays of the shape-first draw (built once per table).
static scc_status ensure_shape_first(scc_table *T)
{
    const int nu = T->hlut.num_unr;
    std::vector<const u128 *> ptr(32, nullptr);
    for (int j = 0; j < nu; j++) {
        if (T->hlut.bal_rank[j] < 0 || T->tj[j] == 0) continue;
        u128 tot;
        scc_status s = table_prefix(T, j, &ptr[j], &tot);
        if (s) return s;
    }
    std::lock_guard<std::mutex> g(T->mu);
    if (T->bal_spre) return SCC_OK;
    const u128 **dp = (const u128 **)T->alloc(32 * sizeof(u128 *));
    u128 *dt = (u128 *)T->alloc(32 * sizeof(u128));
    if (!dp || !dt) return set_error(SCC_ENOMEM, "shape-first tables");
    std::vector<u128> tj(32, 0);
    for (int j = 0; j < nu; j++) tj[j] = T->hlut.bal_rank[j] >= 0 ? T->tj[j] : 0;
    HIP_TRY(hipMemcpyAsync(dp, ptr.data(), 32 * sizeof(u128 *), hipMemcpyHostToDevice, T->stream));
    HIP_TRY(hipMemcpyAsync(dt, tj.data(), 32 * sizeof(u128), hipMemcpyHostToDevice, T->stream));
    HIP_TRY(hipStreamSynchronize(T->stream));
    T->bal_spre = dp;
    T->bal_stj = dt;
    return SCC_OK;
}

// The sampling arguments from structures that already exist: EINVAL (with the
// reason) when a running sum the draw needs has not been built yet.
static scc_status sampling_args(scc_table *T, int shape, SampleArgs *out)
{
    const bool bal = T->rooting == SCC_ROOT_BALANCED;
    const u128 *pre = nullptr;
    u128 total = 0;
    int mode = 0;
    const uint8_t *A_ecol = nullptr;
    if (bal && shape == T->hlut.star_unr) {
        mode = 2;
        pre = T->star_pre;
        total = T->stars;
        if (total == 0) return set_error(SCC_EEMPTY, "no %d-star to sample", T->k);
    } else if (bal && shape < 0) {
        mode = 1;
        total = T->t;
        if (total == 0) return set_error(SCC_EEMPTY, "no colourful %d-treelet to sample", T->k);
        std::lock_guard<std::mutex> g(T->mu);
        if (!T->bal_spre) return set_error(SCC_EINVAL, "the shape-first running sums are not built");
    } else if (shape < 0) {
        pre = T->pre;
        total = T->root_total;
        if (total == 0) return set_error(SCC_EEMPTY, "no colourful %d-treelet to sample", T->k);
    } else {
        std::lock_guard<std::mutex> g(T->mu);
        auto it = T->pre_shape.find(shape);
        if (it == T->pre_shape.end()) return set_error(SCC_EINVAL, "the running sums of shape %d are not built", shape);
        pre = it->second;
        total = T->tot_shape[shape];
        if (total == 0) return set_error(SCC_EEMPTY, "no colourful %d-treelet to sample", T->k);
    }
    {
        std::lock_guard<std::mutex> g(T->hub_mu);
        if (!T->hubpre_ready && !T->hub_host.empty()) return set_error(SCC_EINVAL, "the hub running sums are not built");
        A_ecol = T->ecol;
    }
    SampleArgs A{};
    A.ecol = A_ecol;
    A.mode = mode;
    A.spre = T->bal_spre;
    A.stj = T->bal_stj;
    A.key_xidx = T->key_xidx; A.nkeys = T->hlut.nkeys;
    if (T->hub_count_pre) { A.hub_index = T->hub_index; A.hub_poff = T->hub_poff; A.hub_pre = T->hub_pre; }
    A.g = GraphView{T->n, T->row_ptr, T->col_idx, T->colors};
    A.L = T->dlut; A.k = T->k; A.shape = shape; A.zero = T->rooting == SCC_ROOT_ZERO;
    for (int h = 2; h <= T->k; h++) A.lev[h] = lview(T->lev[h]);
    for (int h = 1; h < T->k; h++) {
        A.Slo[h] = T->S[h].lo; A.Shi[h] = T->S[h].hi; A.Shrow[h] = T->S[h].hrow; A.M[h] = T->S[h].M;
    }
    A.pre = pre; A.total = total;
    *out = A;
    return SCC_OK;
}

scc_status prepare_sampling(scc_table *T, int shape, SampleArgs *out)
{
    const bool bal = T->rooting == SCC_ROOT_BALANCED;
    scc_status s = SCC_OK;
    if (bal && shape == T->hlut.star_unr) {
        if (T->stars == 0) return set_error(SCC_EEMPTY, "no %d-star to sample", T->k);
    } else if (bal && shape < 0) {
        if (T->t == 0) return set_error(SCC_EEMPTY, "no colourful %d-treelet to sample", T->k);
        s = ensure_shape_first(T);
    } else {
        const u128 *pre = nullptr;
        u128 total = 0;
        s = table_prefix(T, shape, &pre, &total);
        if (!s && total == 0) return set_error(SCC_EEMPTY, "no colourful %d-treelet to sample", T->k);
    }
    if (s) return s;
    s = ensure_hub_prefix(T);
    if (!s) s = ensure_edge_colours(T);
    if (s) return s;
    return sampling_args(T, shape, out);
}

scc_status prepare_all_sampling(scc_table *T)
{
    SampleArgs A;
    for (int shape = -1; shape < T->hlut.num_unr; shape++) {
        if (sample_weight(T, shape) == 0) continue;
        scc_status s = prepare_sampling(T, shape, &A);
        if (s && s != SCC_EEMPTY) return s;
    }
    return SCC_OK;
}

void launch_serve_sample(const SampleArgs *args, const ServeChunk *ch, const int64_t *cend, int nch, int64_t total,
                         int *err, int grid, hipStream_t st)
{
    if (total <= 0 || nch <= 0) return;
    hipLaunchKernelGGL(k_serve_sample, dim3((unsigned)std::min<int64_t>(total, grid)), dim3(WAVE), 0, st, args, ch, cend,
                       nch, total, err);
}

extern "C" scc_status scc_sample(const scc_table *tc, int32_t shape, int64_t n, uint64_t seed,
                                 uint64_t stream_id, uint64_t first_index, int32_t *out_verts,
                                 int8_t *out_parent, void *stream)
{
    scc_table *T = const_cast<scc_table *>(tc);
    if (!T) return set_error(SCC_EINVAL, "table NULL");
    if (n < 0) return set_error(SCC_EINVAL, "n < 0");
    if (shape < -1 || shape >= T->hlut.num_unr) return set_error(SCC_EINVAL, "shape %d out of range", shape);
    if (n == 0) return SCC_OK;
    if (!out_verts || !out_parent) return set_error(SCC_EINVAL, "output NULL");
    SampleArgs A;
    scc_status s = prepare_sampling(T, shape, &A);
    if (s) return s;
    hipStream_t st = stream ? (hipStream_t)stream : T->stream;
    int *err = (int *)T->mem.get(16);
    if (!err) return set_error(SCC_ENOMEM, "sample flags");
    A.seed = seed; A.stream = stream_id; A.first = first_index;
    A.nsamp = n; A.verts = out_verts; A.par = out_parent; A.err = err;
    hipError_t e = hipMemsetAsync(err, 0, 4, st);
    const int64_t grid = std::min<int64_t>(n, (int64_t)1 << 20);
    hipLaunchKernelGGL(k_sample, dim3((unsigned)grid), dim3(WAVE), 0, st, A);
    int herr = 0;
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    T->mem.put(err);
    if (e != hipSuccess) return set_error(SCC_EDEVICE, "sample: %s", hipGetErrorString(e));
    if (herr) return set_error(SCC_EDEVICE, "internal: a sample draw fell off its list (%d)", herr);
    return SCC_OK;
}

// ---------------------------------------------------------------------------
// The allocation-free sampling entry point. Its only device scratch, the error
// flags of one call, is this file-scope array: each GPU holds one copy for the
// life of the process. Host code never uses the array's name as an address:
// the device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device (with that device current) on the first call there.
// ---------------------------------------------------------------------------
constexpr int NOALLOC_MAX_DEVICES = 64;
constexpr size_t NOALLOC_SCRATCH_BYTES = 256;   // the maximum: one call's flags, whatever n
static __device__ __align__(256) int scratch[NOALLOC_SCRATCH_BYTES / sizeof(int)];

static std::mutex g_scratch_mu;
static int *g_scratch_ptr[NOALLOC_MAX_DEVICES];   // device address of each GPU's copy, or null

static scc_status scratch_of_current_device(int **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return set_error(SCC_EDEVICE, "no usable current device (%d)", dev);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(SCC_EDEVICE, "scratch address on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = (int *)p;
    }
    *out = g_scratch_ptr[dev];
    return SCC_OK;
}

// clears the flags (a kernel, not a memset node, so that capture records it as one)
__global__ void k_clear_flags(int *flags, int n)
{
    if ((int)threadIdx.x < n) flags[threadIdx.x] = 0;
}

extern "C" scc_status scc_sample_noalloc(const scc_table *tc, int32_t shape, int64_t n, uint64_t seed,
                                         uint64_t stream_id, uint64_t first_index, int32_t *out_verts,
                                         int8_t *out_parent, void *stream)
{
    scc_table *T = const_cast<scc_table *>(tc);
    if (!T) return set_error(SCC_EINVAL, "table NULL");
    if (n < 0) return set_error(SCC_EINVAL, "n < 0");
    if (shape < -1 || shape >= T->hlut.num_unr) return set_error(SCC_EINVAL, "shape %d out of range", shape);
    if (n == 0) return SCC_OK;
    if (!out_verts || !out_parent) return set_error(SCC_EINVAL, "output NULL");
    SampleArgs A;
    scc_status s = sampling_args(T, shape, &A);
    if (s) return s;
    int *flags = nullptr;
    s = scratch_of_current_device(&flags);
    if (s) return s;
    hipStream_t st = stream ? (hipStream_t)stream : T->stream;
    A.seed = seed; A.stream = stream_id; A.first = first_index;
    A.nsamp = n; A.verts = out_verts; A.par = out_parent; A.err = flags;
    hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(WAVE), 0, st, flags, 1);
    const int64_t grid = std::min<int64_t>(n, (int64_t)1 << 20);
    hipLaunchKernelGGL(k_sample, dim3((unsigned)grid), dim3(WAVE), 0, st, A);
    int herr = 0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&herr, flags, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return set_error(SCC_EDEVICE, "sample: %s", hipGetErrorString(e));
    if (herr) return set_error(SCC_EDEVICE, "internal: a sample draw fell off its list (%d)", herr);
    return SCC_OK;
}

extern "C" scc_status scc_occ(const scc_table *T, int64_t v, int32_t key, uint64_t out[2])
{
    if (!T || !out) return set_error(SCC_EINVAL, "NULL argument");
    if (v < 0 || v >= T->n) return set_error(SCC_EINVAL, "vertex out of range");
    if (key >= T->hlut.nkeys || key < -1) return set_error(SCC_EINVAL, "key out of range");
    int h = 1;
    if (key >= 0)
        while (h < T->k && key >= T->hlut.off[h + 1]) h++;
    u128 *d = (u128 *)const_cast<scc_table *>(T)->mem.get(16);
    if (!d) return set_error(SCC_ENOMEM, "occ");
    GraphView g{T->n, T->row_ptr, T->col_idx, T->colors};
    hipLaunchKernelGGL(k_occ, dim3(1), dim3(WAVE), 0, T->stream, g, T->dlut, lview(T->lev[h]), h, v, key, T->eta, d);
    u128 r = 0;
    hipError_t e = hipMemcpyAsync(&r, d, 16, hipMemcpyDeviceToHost, T->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(T->stream);
    const_cast<scc_table *>(T)->mem.put(d);
    if (e != hipSuccess) return set_error(SCC_EDEVICE, "occ: %s", hipGetErrorString(e));
    out[0] = lo64(r);
    out[1] = hi64(r);
    return SCC_OK;
}

extern "C" scc_status scc_export_level(const scc_table *tc, int h, int64_t *nnz_out, int64_t *off,
                                       uint16_t *key, uint64_t *lo, uint64_t *hi, void *stream)
{
    scc_table *T = const_cast<scc_table *>(tc);
    if (!T) return set_error(SCC_EINVAL, "table NULL");
    if (h < 1 || h > T->k) return set_error(SCC_EINVAL, "level %d out of range", h);
    const int64_t nnz = T->lev[h].nnz;
    if (nnz_out) *nnz_out = nnz;
    if (!off) return SCC_OK;
    const int64_t n = T->n;
    hipStream_t st = stream ? (hipStream_t)stream : T->stream;
    if (n == 0) {
        int64_t z = 0;
        HIP_TRY(hipMemcpyAsync(off, &z, 8, hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
        return SCC_OK;
    }
    uint64_t *len = (uint64_t *)T->mem.get((size_t)n * 8);
    if (!len) return set_error(SCC_ENOMEM, "export scratch");
    hipLaunchKernelGGL(k_len, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, T->lev[h].loc, h == 1, T->colors, len);
    hipStream_t keep = T->stream;
    T->stream = st;
    scc_status s = scan_u64(T, len, len, n);
    T->stream = keep;
    if (s) { T->mem.put(len); return s; }
    hipLaunchKernelGGL(k_export, dim3((unsigned)n), dim3(WAVE), 0, st, n, lview(T->lev[h]), h == 1, T->colors, len,
                       off, key, lo, hi);
    hipError_t e = hipStreamSynchronize(st);
    T->mem.put(len);
    if (e != hipSuccess) return set_error(SCC_EDEVICE, "export: %s", hipGetErrorString(e));
    return SCC_OK;
}
