// The build-up phase on the GPU (Sec. 2.1, Eq. (1)).
//
// Level h >= 2 of the table is computed in four steps per level:
//   bound   M_{h-1}(v) = sum_{u~v} N_{h-1}(u), the per-vertex bound that picks
//           64- or 128-bit arithmetic before any count is formed;
//   gather  S_{h-1}(T''_{C''}, v) = sum_{u~v} c(T''_{C''}, u): the neighbours'
//           compacted records are streamed and added into a dense per-vertex
//           accumulator in LDS, indexed by (rank T'', colex of C'' without c_v);
//   combine c(T_C, v) = (1/beta_T) sum_{C'} c(T'_{C'}, v) S(T''_{C \ C'}, v)
//           for every (T, C) with c_v in C, from v's own lower levels and
//           neighbour sums staged in LDS; non-zero results are compacted with
//           wave ballots into fixed-capacity per-vertex slots;
//   pack    an exclusive scan of record sizes and a copy into one vertex-ordered
//           pool of succinct records (u16 keys, then low words, then high words
//           for 128-bit vertices) (Sec. 3.2 "Count tables").
// Level k is kept at colour-0 vertices under zero-rooting (Sec. 3.4).
#include <algorithm>
#include <chrono>
#include <cstring>

#include "table.hpp"

namespace {

constexpr int MAXR = 7;    // ceil(max W_h / 64): W_h <= 420 for k <= 8

// ---------------------------------------------------------------------------
// CSR and colour validation (Sec. 1.3: simple undirected graph)
// ---------------------------------------------------------------------------
__global__ void k_validate(GraphView g, int k, int *err)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    int bad = 0;
    if (g.colors[v] >= k) bad |= 1;
    int64_t a = g.row_ptr[v], b = g.row_ptr[v + 1];
    if (b < a) bad |= 2;
    for (int64_t e = a; e < b && !(bad & 2); e++) {
        int32_t u = g.col_idx[e];
        if (u < 0 || u >= g.n || u == v) { bad |= 4; break; }
        if (e > a && g.col_idx[e - 1] >= u) { bad |= 8; break; }
        int64_t lo = g.row_ptr[u], hi = g.row_ptr[u + 1];
        int found = 0;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            int32_t w = g.col_idx[mid];
            if (w == v) { found = 1; break; }
            if (w < v) lo = mid + 1; else hi = mid;
        }
        if (!found) { bad |= 16; break; }
    }
    if (bad) atomicOr(err, bad);
}

// ---------------------------------------------------------------------------
// Level-1 neighbour sums: S_1(v)[j] = number of neighbours of colour j != c_v
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(WAVE) k_gather1(GraphView g, int k, uint64_t *S1, u128 *M1)
{
    __shared__ unsigned cnt[SCC_KMAX];
    const int64_t v = blockIdx.x;
    const int lane = threadIdx.x;
    const int cv = g.colors[v];
    if (lane < SCC_KMAX) cnt[lane] = 0;
    __syncthreads();
    const int64_t a = g.row_ptr[v], b = g.row_ptr[v + 1];
    for (int64_t e = a + lane; e < b; e += WAVE) {
        int cu = g.colors[g.col_idx[e]];
        if (cu != cv) atomicAdd(&cnt[cu], 1u);
    }
    __syncthreads();
    if (lane < k && lane != cv) {
        // compressed index of the singleton {lane}: its rank among 1-subsets = position
        int pos = lane < cv ? lane : lane - 1;
        S1[v * (k - 1) + pos] = cnt[lane];
    }
    if (lane == 0) M1[v] = (u128)(b - a);
}

// ---------------------------------------------------------------------------
// Bound pass for level h' = hs (>= 2): M_hs(v) = sum_{u~v} N_hs(u) (saturating),
// whether any M needs 128 bits, whether any vertex of level hs+1 will need
// 128-bit counts, and the gather's algorithmic byte count.
// ---------------------------------------------------------------------------
struct BoundArgs {
    GraphView g;
    int hs, k, zero_next;          // zero_next: level hs+1 == k under zero-rooting
    int rows_zero;                 // gather rows restricted to colour-0 vertices
    LevelView L;                   // level hs
    const u128 *Nlev[SCC_KMAX + 1];
    const u128 *Mlev[SCC_KMAX + 1];
    u128 *Mout;
    int WS;                        // entries of S_hs per vertex
    unsigned long long *flags;     // [0] any M >= 2^64, [1] any U >= 2^64, [2] any U saturated, [3] bytes
};

__global__ void __launch_bounds__(WAVE) k_bound(BoundArgs A)
{
    const int64_t v = blockIdx.x;
    const int lane = threadIdx.x;
    const int cv = A.g.colors[v];
    const int64_t a = A.g.row_ptr[v], b = A.g.row_ptr[v + 1];
    u128 m = 0;
    uint64_t bytes = 0;
    for (int64_t e = a + lane; e < b; e += WAVE) {
        int32_t u = A.g.col_idx[e];
        m = sat_add(m, A.L.N[u]);
        uint32_t mm = A.L.meta[u];
        bytes += (uint64_t)META_LEN(mm) * (META_WIDE(mm) ? 18u : 10u);
    }
    m = wave_satsum128(m);
    bytes = wave_sum64(bytes);
    if (lane != 0) return;
    A.Mout[v] = m;
    if (hi64(m)) atomicOr(&A.flags[0], 1ull);
    const bool row = !A.rows_zero || cv == 0;
    if (row) atomicAdd(&A.flags[3], bytes + 4ull * (uint64_t)(b - a) + (uint64_t)A.WS * (hi64(m) ? 16u : 8u));
    // bound of level hs + 1 at v
    if (A.zero_next && cv != 0) return;
    const int h = A.hs + 1;
    u128 U = 0;
    for (int hp = 1; hp < h; hp++) {
        u128 Nv = hp == 1 ? (u128)1 : A.Nlev[hp][v];
        u128 Mv = (h - hp == A.hs) ? m : A.Mlev[h - hp][v];
        U = sat_add(U, sat_mul(Nv, Mv));
    }
    if (U == ~(u128)0) atomicOr(&A.flags[2], 1ull);
    if (hi64(U)) atomicOr(&A.flags[1], 1ull);
}

// ---------------------------------------------------------------------------
// Gather (the DP join): S_hs(v) = sum over neighbours of their level-hs records
// ---------------------------------------------------------------------------
struct GatherArgs {
    GraphView g;
    int k, nkeys, WS, rows_zero;
    LevelView L;
    const u128 *M;                 // M_hs
    const int16_t *key_sidx;       // [k * nkeys]
    uint64_t *Slo, *Shi;           // [n * WS]
};

__global__ void __launch_bounds__(WAVE) k_gather(GatherArgs A)
{
    extern __shared__ uint64_t sm[];
    const int64_t v = blockIdx.x;
    const int lane = threadIdx.x;
    const int cv = A.g.colors[v];
    if (A.rows_zero && cv != 0) return;
    const int WS = A.WS;
    uint64_t *acc_lo = sm;
    uint64_t *acc_hi = sm + WS;
    const bool wideS = hi64(A.M[v]) != 0;
    for (int i = lane; i < WS; i += WAVE) { acc_lo[i] = 0; acc_hi[i] = 0; }
    __syncthreads();
    const int16_t *sidx = A.key_sidx + (size_t)cv * A.nkeys;
    const int64_t a = A.g.row_ptr[v], b = A.g.row_ptr[v + 1];
    for (int64_t base = a; base < b; base += WAVE) {
        const int64_t e = base + lane;
        uint32_t len = 0, meta = 0;
        uint64_t off = 0;
        if (e < b) {
            int32_t u = A.g.col_idx[e];
            meta = A.L.meta[u];
            len = META_LEN(meta);
            if (len) off = A.L.off[u];
        }
        const uint32_t incl = wave_incl_scan32(len);
        const uint32_t total = __shfl(incl, WAVE - 1, WAVE);
        // entries of this chunk of neighbours, flattened over the lanes
        for (uint32_t p0 = 0; p0 < total; p0 += WAVE) {
            const uint32_t p = p0 + lane;
            // owner neighbour j: number of lanes whose inclusive count is <= p
            // (fixed six steps, so every lane takes part in every shuffle)
            int j = 0;
#pragma unroll
            for (int step = WAVE / 2; step >= 1; step >>= 1) {
                uint32_t x = __shfl(incl, j + step - 1, WAVE);
                if (x <= p) j += step;
            }
            if (j > WAVE - 1) j = WAVE - 1;
            const uint32_t incl_j = __shfl(incl, j, WAVE);
            const uint32_t meta_j = __shfl(meta, j, WAVE);
            const uint64_t off_j = shfl64(off, j);
            if (p < total) {
                const uint32_t len_j = META_LEN(meta_j);
                const uint32_t ei = p - (incl_j - len_j);
                const uint64_t *rec = A.L.pool + off_j;
                const uint32_t kw = key_words(len_j);
                const uint32_t key = ((const uint16_t *)rec)[ei];
                const uint64_t cl = rec[kw + ei];
                const int s = sidx[key];
                if (s >= 0) {
                    if (!wideS) {
                        atomicAdd((unsigned long long *)&acc_lo[s], (unsigned long long)cl);
                    } else {
                        const uint64_t ch = META_WIDE(meta_j) ? rec[kw + len_j + ei] : 0;
                        unsigned long long old = atomicAdd((unsigned long long *)&acc_lo[s], (unsigned long long)cl);
                        uint64_t carry = (old + cl) < old ? 1u : 0u;
                        if (ch + carry) atomicAdd((unsigned long long *)&acc_hi[s], (unsigned long long)(ch + carry));
                    }
                }
            }
        }
    }
    __syncthreads();
    uint64_t *Slo = A.Slo + (size_t)v * WS;
    for (int i = lane; i < WS; i += WAVE) Slo[i] = acc_lo[i];
    if (wideS) {
        uint64_t *Shi = A.Shi + (size_t)v * WS;
        for (int i = lane; i < WS; i += WAVE) Shi[i] = acc_hi[i];
    }
}

// ---------------------------------------------------------------------------
// Combine: Eq. (1) with the neighbour sum already formed
// ---------------------------------------------------------------------------
struct CombineArgs {
    GraphView g;
    const DevLut *L;
    int h, zero_only, max_bits;
    LevelView lev[SCC_KMAX + 1];          // own levels 2..h-1
    const uint64_t *Slo[SCC_KMAX + 1];    // neighbour sums 1..h-1
    const uint64_t *Shi[SCC_KMAX + 1];
    const u128 *M[SCC_KMAX + 1];
    const int16_t *key_xidx;              // [k * nkeys]
    int W;                                // slot capacity = W_h
    uint16_t *slot_key;
    uint64_t *slot_lo, *slot_hi;          // slot_hi may be null (no wide vertex)
    uint32_t *meta;
    u128 *Nout;
    int *err;                             // [0]: overflow
};

__global__ void __launch_bounds__(WAVE) k_combine(CombineArgs A)
{
    extern __shared__ uint64_t sm[];
    const DevLut &L = *A.L;
    const int64_t v = blockIdx.x;
    const int lane = threadIdx.x;
    const int h = A.h;
    const int cv = A.g.colors[v];
    if (A.zero_only && cv != 0) {
        if (lane == 0) { A.meta[v] = 0; A.Nout[v] = 0; }
        return;
    }
    // per-vertex bound: U >= sum over (T, C) of beta_T c(T_C, v) >= every partial sum
    u128 U = 0;
    for (int hp = 1; hp < h; hp++) {
        u128 Nv = hp == 1 ? (u128)1 : A.lev[hp].N[v];
        U = sat_add(U, sat_mul(Nv, A.M[h - hp][v]));
    }
    if (U == ~(u128)0 || bitlen128(U) > A.max_bits) {
        if (lane == 0) { atomicOr(A.err, 1); A.meta[v] = 0; A.Nout[v] = 0; }
        return;
    }
    const bool wide = hi64(U) != 0;
    const int XT = L.xoff[h], ST = L.soff[h];
    uint64_t *Xlo = sm, *Xhi = sm + XT, *Slo = sm + 2 * XT, *Shi = sm + 2 * XT + ST;
    for (int i = lane; i < XT; i += WAVE) { Xlo[i] = 0; Xhi[i] = 0; }
    __syncthreads();
    if (lane == 0) Xlo[L.xoff[1]] = 1;   // level 1: the single node, coloured c_v
    const int16_t *xidx = A.key_xidx + (size_t)cv * L.nkeys;
    for (int hp = 2; hp < h; hp++) {
        const LevelView &Lv = A.lev[hp];
        const uint32_t m = Lv.meta[v], len = META_LEN(m);
        if (!len) continue;
        const uint64_t *rec = Lv.pool + Lv.off[v];
        const uint32_t kw = key_words(len);
        for (uint32_t e = lane; e < len; e += WAVE) {
            uint32_t key = ((const uint16_t *)rec)[e];
            int x = L.xoff[hp] + xidx[key];
            Xlo[x] = rec[kw + e];
            Xhi[x] = META_WIDE(m) ? rec[kw + len + e] : 0;
        }
    }
    for (int hs = 1; hs < h; hs++) {
        const int ws = L.WS[hs];
        const uint64_t *gl = A.Slo[hs] + (size_t)v * ws;
        const bool sw = hi64(A.M[hs][v]) != 0;
        const uint64_t *gh = sw ? A.Shi[hs] + (size_t)v * ws : nullptr;
        for (int i = lane; i < ws; i += WAVE) {
            Slo[L.soff[hs] + i] = gl[i];
            Shi[L.soff[hs] + i] = sw ? gh[i] : 0;
        }
    }
    __syncthreads();

    const int Wh = L.W[h];
    const int nD = L.bk1[h - 1];
    u128 val[MAXR];
#pragma unroll
    for (int r = 0; r < MAXR; r++) {
        val[r] = 0;
        const int o = r * WAVE + lane;
        if (o < Wh) {
            const int t = o / nD, dc = o - t * nD;
            const int hp = L.dec_hp[h][t], hpp = h - hp;
            const int xb = L.xoff[hp] + L.dec_a[h][t] * L.bk1[hp - 1];
            const int sb = L.soff[hpp] + L.dec_b[h][t] * L.bk1[hpp];
            // number of splits = binom(h-1, hp-1)
            int nsplit = 1;
            for (int i = 1; i <= hp - 1; i++) nsplit = nsplit * (h - 1 - (hp - 1) + i) / i;
            const int tb = L.term_base[h][hp] + dc * nsplit;
            u128 acc = 0;
            if (!wide) {
                uint64_t a64 = 0;
                for (int i = 0; i < nsplit; i++)
                    a64 += Xlo[xb + L.term_x[tb + i]] * Slo[sb + L.term_s[tb + i]];
                acc = a64;
            } else {
                for (int i = 0; i < nsplit; i++) {
                    const int xi = xb + L.term_x[tb + i], si = sb + L.term_s[tb + i];
                    u128 x = mk128(Xlo[xi], Xhi[xi]), s = mk128(Slo[si], Shi[si]);
                    acc += x * s;
                }
            }
            const int beta = L.dec_beta[h][t];
            val[r] = beta == 1 ? acc : div_small(acc, (uint32_t)beta);
        }
    }
    // compaction into v's slot: ballot + prefix count keeps ascending key order
    uint32_t cnt = 0;
    u128 nsum = 0;
    uint16_t *sk = A.slot_key + (size_t)v * A.W;
    uint64_t *sl = A.slot_lo + (size_t)v * A.W;
    uint64_t *sh = wide ? A.slot_hi + (size_t)v * A.W : nullptr;
#pragma unroll
    for (int r = 0; r < MAXR; r++) {
        const int o = r * WAVE + lane;
        const bool nz = o < Wh && val[r] != 0;
        const uint64_t bal = __ballot(nz);
        if (nz) {
            const uint32_t pos = cnt + (uint32_t)__popcll(bal & lanemask_lt());
            const int t = o / nD, dc = o - t * nD;
            const uint32_t D = L.mask_s[h - 1][dc];
            const uint32_t C = expand_in(D, cv) | (1u << cv);
            sk[pos] = (uint16_t)(L.off[h] + t * L.bk[h] + L.colex_k[C]);
            sl[pos] = lo64(val[r]);
            if (wide) sh[pos] = hi64(val[r]);
            nsum += val[r];
        }
        cnt += (uint32_t)__popcll(bal);
    }
    nsum = wave_sum128(nsum);
    if (lane == 0) {
        A.meta[v] = cnt | (wide ? 0x80000000u : 0u);
        A.Nout[v] = nsum;
    }
}

// stored entries and 128-bit vertices of a level
__global__ void k_meta_sum(int64_t n, const uint32_t *meta, unsigned long long *out)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t len = 0, wide = 0;
    if (v < n) {
        const uint32_t m = meta[v];
        len = META_LEN(m);
        wide = META_WIDE(m);
    }
    len = wave_sum64(len);
    wide = wave_sum64(wide);
    if (lane_id() == 0 && (len || wide)) {
        atomicAdd(&out[0], (unsigned long long)len);
        atomicAdd(&out[1], (unsigned long long)wide);
    }
}

// record size in 64-bit words
__global__ void k_words(int64_t n, const uint32_t *meta, uint64_t *words)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    uint32_t m = meta[v], len = META_LEN(m);
    words[v] = len ? (uint64_t)key_words(len) + (uint64_t)len * (META_WIDE(m) ? 2u : 1u) : 0;
}

// copy each vertex's slot into the packed pool at its offset
__global__ void __launch_bounds__(WAVE) k_pack(int64_t n, int W, const uint32_t *meta, const uint64_t *off_incl,
                                               const uint16_t *slot_key, const uint64_t *slot_lo,
                                               const uint64_t *slot_hi, uint64_t *pool, uint64_t *off)
{
    const int64_t v = blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t m = meta[v], len = META_LEN(m);
    const uint32_t words = len ? key_words(len) + len * (META_WIDE(m) ? 2u : 1u) : 0;
    const uint64_t start = off_incl[v] - words;
    if (lane == 0) off[v] = start;
    if (!len) return;
    uint64_t *rec = pool + start;
    const uint32_t kw = key_words(len);
    uint16_t *keys = (uint16_t *)rec;
    for (uint32_t e = lane; e < kw * 4; e += WAVE) keys[e] = e < len ? slot_key[(size_t)v * W + e] : 0;
    for (uint32_t e = lane; e < len; e += WAVE) rec[kw + e] = slot_lo[(size_t)v * W + e];
    if (META_WIDE(m))
        for (uint32_t e = lane; e < len; e += WAVE) rec[kw + len + e] = slot_hi[(size_t)v * W + e];
}

// ---------------------------------------------------------------------------
// Level-k totals: eta_v (all shapes) and per-block partial sums per unrooted shape
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_totals(GraphView g, const DevLut *Lp, LevelView Lk, int zero_only, u128 *eta, u128 *part)
{
    __shared__ u128 wpart[256 / WAVE][32];
    const DevLut &L = *Lp;
    const int tid = threadIdx.x;
    const int nu = L.num_unr;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + tid;
    uint32_t len = 0, m = 0;
    const uint64_t *rec = nullptr;
    if (v < g.n && (!zero_only || g.colors[v] == 0)) {
        m = Lk.meta[v];
        len = META_LEN(m);
        if (len) rec = Lk.pool + Lk.off[v];
    }
    u128 e = 0;
    const uint32_t kw = key_words(len);
    for (int j = 0; j < nu; j++) {
        u128 sj = 0;
        for (uint32_t q = 0; q < len; q++) {
            const uint32_t key = ((const uint16_t *)rec)[q];
            const int t = (int)(key - L.off[L.k]) / L.bk[L.k];
            if (L.unr_of[t] == j) sj += mk128(rec[kw + q], META_WIDE(m) ? rec[kw + len + q] : 0);
        }
        e += sj;
        sj = wave_sum128(sj);
        if (lane_id() == 0) wpart[tid / WAVE][j] = sj;
    }
    if (v < g.n) eta[v] = e;
    __syncthreads();
    if (tid < nu) {
        u128 s = 0;
        for (int w = 0; w < (int)(blockDim.x / WAVE); w++) s += wpart[w][tid];
        part[(size_t)blockIdx.x * 32 + tid] = s;
    }
}

__global__ void k_reduce_parts(const u128 *part, int nb, int nu, u128 *out)
{
    const int j = threadIdx.x;
    if (j >= nu) return;
    u128 s = 0;
    for (int b = 0; b < nb; b++) s += part[(size_t)b * 32 + j];
    out[j] = s;
}

__global__ void k_eta_shape(GraphView g, const DevLut *Lp, LevelView Lk, int zero_only, int shape, u128 *eta)
{
    const DevLut &L = *Lp;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    u128 e = 0;
    if (!zero_only || g.colors[v] == 0) {
        const uint32_t m = Lk.meta[v], len = META_LEN(m);
        if (len) {
            const uint64_t *rec = Lk.pool + Lk.off[v];
            const uint32_t kw = key_words(len);
            for (uint32_t q = 0; q < len; q++) {
                const uint32_t key = ((const uint16_t *)rec)[q];
                const int t = (key - L.off[L.k]) / L.bk[L.k];
                if (L.unr_of[t] == shape) e += mk128(rec[kw + q], META_WIDE(m) ? rec[kw + len + q] : 0);
            }
        }
    }
    eta[v] = e;
}

// ---------------------------------------------------------------------------
// Inclusive scans (u128 and u64): block sums, a one-block scan of the sums,
// then each block scans its tile and adds its prefix.
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 256, SCAN_I = 4, SCAN_TILE = SCAN_T * SCAN_I;

template <typename T>
__device__ T block_incl_scan(T x, T *sh)
{
    // sh: SCAN_T / WAVE entries
    const int lane = lane_id(), w = threadIdx.x / WAVE;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T y;
        if constexpr (sizeof(T) == 16) {
            uint64_t l = (uint64_t)__shfl_up((unsigned long long)lo64((u128)x), d, WAVE);
            uint64_t hh = (uint64_t)__shfl_up((unsigned long long)hi64((u128)x), d, WAVE);
            y = (T)mk128(l, hh);
        } else {
            y = (T)__shfl_up((unsigned long long)x, d, WAVE);
        }
        if (lane >= d) x += y;
    }
    if (lane == WAVE - 1) sh[w] = x;
    __syncthreads();
    T pre = 0;
    for (int i = 0; i < w; i++) pre += sh[i];
    __syncthreads();
    return x + pre;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_T) k_scan_sums(const T *in, int64_t n, T *bsum)
{
    __shared__ T sh[SCAN_T / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    T s = 0;
    for (int i = 0; i < SCAN_I; i++) {
        int64_t idx = base + (int64_t)threadIdx.x * SCAN_I + i;
        if (idx < n) s += in[idx];
    }
    T incl = block_incl_scan<T>(s, sh);
    if (threadIdx.x == SCAN_T - 1) bsum[blockIdx.x] = incl;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_T) k_scan_top(T *bsum, int64_t nb)
{
    // exclusive scan of the block sums, one tile at a time
    __shared__ T sh[SCAN_T / WAVE];
    __shared__ T carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += SCAN_T) {
        int64_t idx = base + threadIdx.x;
        T x = idx < nb ? bsum[idx] : (T)0;
        T incl = block_incl_scan<T>(x, sh);
        T c = carry;
        if (idx < nb) bsum[idx] = c + incl - x;
        __syncthreads();
        if (threadIdx.x == SCAN_T - 1) carry = c + incl;
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(SCAN_T) k_scan_apply(const T *in, T *out, int64_t n, const T *bexcl)
{
    __shared__ T sh[SCAN_T / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_I;
    T v[SCAN_I];
    T s = 0;
    for (int i = 0; i < SCAN_I; i++) {
        v[i] = (base + i < n) ? in[base + i] : (T)0;
        s += v[i];
    }
    T incl = block_incl_scan<T>(s, sh);
    T run = bexcl[blockIdx.x] + incl - s;
    for (int i = 0; i < SCAN_I; i++) {
        run += v[i];
        if (base + i < n) out[base + i] = run;
    }
}

template <typename T>
scc_status scan_incl(scc_table *T_, const T *in, T *out, int64_t n)
{
    if (n <= 0) return SCC_OK;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    T *bsum = (T *)T_->mem.get(nb * sizeof(T));
    if (!bsum) return set_error(SCC_ENOMEM, "scan scratch");
    hipLaunchKernelGGL(k_scan_sums<T>, dim3((unsigned)nb), dim3(SCAN_T), 0, T_->stream, in, n, bsum);
    hipLaunchKernelGGL(k_scan_top<T>, dim3(1), dim3(SCAN_T), 0, T_->stream, bsum, nb);
    hipLaunchKernelGGL(k_scan_apply<T>, dim3((unsigned)nb), dim3(SCAN_T), 0, T_->stream, in, out, n, bsum);
    hipError_t e = hipStreamSynchronize(T_->stream);
    T_->mem.put(bsum);
    if (e != hipSuccess) return set_error(SCC_EDEVICE, "scan: %s", hipGetErrorString(e));
    return SCC_OK;
}

LevelView view(const TableLevel &l)
{
    return LevelView{l.pool, l.off, l.meta, l.N};
}

}  // namespace

scc_status scan_u128(scc_table *T, const u128 *in, u128 *out, int64_t n) { return scan_incl<u128>(T, in, out, n); }
scc_status scan_u64(scc_table *T, const uint64_t *in, uint64_t *out, int64_t n) { return scan_incl<uint64_t>(T, in, out, n); }
scc_status scan_u32(scc_table *T, const uint32_t *in, uint32_t *out, int64_t n) { return scan_incl<uint32_t>(T, in, out, n); }

void launch_eta_shape(scc_table *T, int shape, u128 *eta)
{
    GraphView g{T->n, T->row_ptr, T->col_idx, T->colors};
    if (T->n)
        hipLaunchKernelGGL(k_eta_shape, dim3((unsigned)((T->n + 255) / 256)), dim3(256), 0, T->stream, g, T->dlut,
                           view(T->lev[T->k]), T->rooting == SCC_ROOT_ZERO ? 1 : 0, shape, eta);
}

// ---------------------------------------------------------------------------
// Host orchestration
// ---------------------------------------------------------------------------
static scc_status build_levels(scc_table *T)
{
    const DevLut &HL = T->hlut;
    const int k = T->k;
    const int64_t n = T->n;
    hipStream_t st = T->stream;
    GraphView g{n, T->row_ptr, T->col_idx, T->colors};
    const bool zero = T->rooting == SCC_ROOT_ZERO;

    unsigned long long *flags = (unsigned long long *)T->mem.get(8 * sizeof(unsigned long long));
    int *err = (int *)T->mem.get(16);
    if (!flags || !err) return set_error(SCC_ENOMEM, "flags");
    struct Guard {
        scc_table *T; void *a, *b;
        ~Guard() { T->mem.put(a); T->mem.put(b); }
    } guard{T, flags, err};

    hipEvent_t e0, e1, g0, g1;
    HIP_TRY(hipEventCreate(&e0)); HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventCreate(&g0)); HIP_TRY(hipEventCreate(&g1));
    struct EvGuard { hipEvent_t a, b, c, d; ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); (void)hipEventDestroy(c); (void)hipEventDestroy(d); } } evg{e0, e1, g0, g1};

    // level 1 neighbour sums
    TableSums &S1 = T->S[1];
    S1.lo = (uint64_t *)T->alloc((size_t)n * (k - 1) * 8);
    S1.M = (u128 *)T->alloc((size_t)n * 16);
    if (!S1.lo || !S1.M) return set_error(SCC_ENOMEM, "level-1 sums");
    HIP_TRY(hipEventRecord(g0, st));
    if (n) hipLaunchKernelGGL(k_gather1, dim3((unsigned)n), dim3(WAVE), 0, st, g, k, S1.lo, S1.M);
    HIP_TRY(hipEventRecord(g1, st));
    HIP_TRY(hipEventSynchronize(g1));
    {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, g0, g1));
        T->gather_ms[1] = ms;
        T->gather_bytes[1] = (double)n * 8.0 + (double)T->nnz_g * 5.0 + (double)n * (k - 1) * 8.0;
        T->level_ms[1] = ms;
    }

    // scratch slots for the combine, sized for the widest level
    int maxW = 0;
    for (int h = 2; h <= k; h++) maxW = std::max(maxW, HL.W[h]);
    uint16_t *slot_key = (uint16_t *)T->mem.get((size_t)n * maxW * 2 + 256);
    uint64_t *slot_lo = (uint64_t *)T->mem.get((size_t)n * maxW * 8 + 256);
    uint64_t *slot_hi = nullptr;
    uint64_t *words = (uint64_t *)T->mem.get((size_t)n * 8 + 256);
    if (!slot_key || !slot_lo || !words) {
        T->mem.put(slot_key); T->mem.put(slot_lo); T->mem.put(words);
        return set_error(SCC_ENOMEM, "combine scratch (%lld bytes)", (long long)n * maxW * 10);
    }
    struct SlotGuard { scc_table *T; void **a, **b, **c, **d; ~SlotGuard() { T->mem.put(*a); T->mem.put(*b); T->mem.put(*c); T->mem.put(*d); } }
        sg{T, (void **)&slot_key, (void **)&slot_lo, (void **)&slot_hi, (void **)&words};

    for (int h = 2; h <= k; h++) {
        const bool last = h == k;
        HIP_TRY(hipEventRecord(e0, st));
        HIP_TRY(hipMemsetAsync(flags, 0, 8 * sizeof(unsigned long long), st));
        HIP_TRY(hipMemsetAsync(err, 0, 16, st));
        const int hs = h - 1;   // neighbour sums needed now
        bool any_wide = false;
        if (hs >= 2) {
            // bound and gather of level hs
            TableSums &Sx = T->S[hs];
            Sx.M = (u128 *)T->alloc((size_t)n * 16);
            if (!Sx.M) return set_error(SCC_ENOMEM, "bounds");
            BoundArgs B{};
            B.g = g; B.hs = hs; B.k = k; B.zero_next = zero && h == k; B.rows_zero = zero && h == k;
            B.L = view(T->lev[hs]);
            for (int q = 2; q < h; q++) B.Nlev[q] = T->lev[q].N;
            for (int q = 1; q < hs; q++) B.Mlev[q] = T->S[q].M;
            B.Mout = Sx.M; B.WS = HL.WS[hs]; B.flags = flags;
            if (n) hipLaunchKernelGGL(k_bound, dim3((unsigned)n), dim3(WAVE), 0, st, B);
            unsigned long long hf[4];
            HIP_TRY(hipMemcpyAsync(hf, flags, sizeof hf, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (hf[2]) return set_error(SCC_EOVERFLOW, "a level-%d count may exceed 128 bits", h);
            any_wide = hf[1] != 0;
            T->gather_bytes[hs] = (double)hf[3];
            const size_t sz = (size_t)n * HL.WS[hs] * 8;
            Sx.lo = (uint64_t *)T->alloc(sz + 8);
            if (!Sx.lo) return set_error(SCC_ENOMEM, "neighbour sums level %d (%zu bytes)", hs, sz);
            if (hf[0]) {
                Sx.hi = (uint64_t *)T->alloc(sz + 8);
                if (!Sx.hi) return set_error(SCC_ENOMEM, "neighbour sums level %d (high words)", hs);
            }
            GatherArgs G{};
            G.g = g; G.k = k; G.nkeys = HL.nkeys; G.WS = HL.WS[hs]; G.rows_zero = zero && h == k;
            G.L = view(T->lev[hs]); G.M = Sx.M; G.key_sidx = T->key_sidx; G.Slo = Sx.lo; G.Shi = Sx.hi;
            HIP_TRY(hipEventRecord(g0, st));
            if (n) hipLaunchKernelGGL(k_gather, dim3((unsigned)n), dim3(WAVE), (size_t)2 * HL.WS[hs] * 8, st, G);
            HIP_TRY(hipEventRecord(g1, st));
        } else {
            // level 2 needs only level-1 sums; its bound is c <= d_v
            any_wide = false;
        }
        if (T->max_bits < 128 && any_wide) {
            // checked per vertex below; a 64-bit table rejects the level
        }
        // combine into slots
        TableLevel &Lv = T->lev[h];
        Lv.meta = (uint32_t *)T->alloc((size_t)n * 4 + 8);
        Lv.N = (u128 *)T->alloc((size_t)n * 16 + 16);
        Lv.off = (uint64_t *)T->alloc((size_t)n * 8 + 8);
        if (!Lv.meta || !Lv.N || !Lv.off) return set_error(SCC_ENOMEM, "level %d metadata", h);
        if (any_wide && !slot_hi) {
            slot_hi = (uint64_t *)T->mem.get((size_t)n * maxW * 8 + 256);
            if (!slot_hi) return set_error(SCC_ENOMEM, "wide combine scratch");
        }
        CombineArgs C{};
        C.g = g; C.L = T->dlut; C.h = h; C.zero_only = zero && last; C.max_bits = T->max_bits;
        for (int q = 2; q < h; q++) C.lev[q] = view(T->lev[q]);
        for (int q = 1; q < h; q++) { C.Slo[q] = T->S[q].lo; C.Shi[q] = T->S[q].hi; C.M[q] = T->S[q].M; }
        C.key_xidx = T->key_xidx; C.W = HL.W[h];
        C.slot_key = slot_key; C.slot_lo = slot_lo; C.slot_hi = slot_hi;
        C.meta = Lv.meta; C.Nout = Lv.N; C.err = err;
        const size_t lds = (size_t)(2 * HL.xoff[h] + 2 * HL.soff[h]) * 8;
        if (n) hipLaunchKernelGGL(k_combine, dim3((unsigned)n), dim3(WAVE), lds, st, C);
        int herr[4];
        HIP_TRY(hipMemcpyAsync(herr, err, sizeof herr, hipMemcpyDeviceToHost, st));
        // record sizes, offsets, pack
        if (n) hipLaunchKernelGGL(k_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, Lv.meta, words);
        HIP_TRY(hipStreamSynchronize(st));
        if (herr[0]) return set_error(SCC_EOVERFLOW, "a level-%d count needs more than %d bits", h, T->max_bits);
        if (hs >= 2) {
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, g0, g1));
            T->gather_ms[hs] = ms;
        }
        scc_status sst = scan_incl<uint64_t>(T, words, words, n);
        if (sst) return sst;
        uint64_t total = 0;
        if (n) {
            HIP_TRY(hipMemcpyAsync(&total, words + (n - 1), 8, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        Lv.pool_words = total;
        Lv.pool = (uint64_t *)T->alloc((size_t)total * 8 + 64);
        if (!Lv.pool) return set_error(SCC_ENOMEM, "level %d pool (%llu words)", h, (unsigned long long)total);
        if (n) hipLaunchKernelGGL(k_pack, dim3((unsigned)n), dim3(WAVE), 0, st, n, HL.W[h], Lv.meta, words,
                                  slot_key, slot_lo, slot_hi, Lv.pool, Lv.off);
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipMemsetAsync(flags, 0, 2 * sizeof(unsigned long long), st));
        if (n) hipLaunchKernelGGL(k_meta_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, Lv.meta, flags);
        unsigned long long cnt2[2];
        HIP_TRY(hipMemcpyAsync(cnt2, flags, sizeof cnt2, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        Lv.nnz = (int64_t)cnt2[0];
        Lv.wide = (int64_t)cnt2[1];
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        T->level_ms[h] = ms;
        HIP_TRY(hipGetLastError());
    }
    return SCC_OK;
}

static scc_status build_totals(scc_table *T)
{
    const int k = T->k;
    const int64_t n = T->n;
    hipStream_t st = T->stream;
    GraphView g{n, T->row_ptr, T->col_idx, T->colors};
    const bool zero = T->rooting == SCC_ROOT_ZERO;
    T->eta = (u128 *)T->alloc((size_t)n * 16 + 16);
    T->pre = (u128 *)T->alloc((size_t)n * 16 + 16);
    const int64_t nb = std::max<int64_t>(1, (n + 255) / 256);
    u128 *part = (u128 *)T->mem.get((size_t)nb * 32 * 16);
    u128 *tjd = (u128 *)T->mem.get(32 * 16);
    if (!T->eta || !T->pre || !part || !tjd) { T->mem.put(part); T->mem.put(tjd); return set_error(SCC_ENOMEM, "totals"); }
    if (n) hipLaunchKernelGGL(k_totals, dim3((unsigned)nb), dim3(256), 0, st, g, T->dlut, view(T->lev[k]), zero ? 1 : 0, T->eta, part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(32), 0, st, part, (int)(n ? nb : 0), T->hlut.num_unr, tjd);
    u128 tj[32];
    hipError_t e = hipMemcpyAsync(tj, tjd, sizeof tj, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    T->mem.put(part);
    T->mem.put(tjd);
    if (e != hipSuccess) return set_error(SCC_EDEVICE, "totals: %s", hipGetErrorString(e));
    scc_status s = scan_u128(T, T->eta, T->pre, n);
    if (s) return s;
    u128 tot = 0;
    if (n) {
        HIP_TRY(hipMemcpyAsync(&tot, T->pre + (n - 1), 16, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    T->root_total = tot;
    for (int j = 0; j < T->hlut.num_unr; j++) T->tj[j] = zero ? tj[j] : tj[j] / (u128)k;
    T->t = zero ? tot : tot / (u128)k;
    return SCC_OK;
}

static scc_status make_key_maps(scc_table *T)
{
    const DevLut &L = T->hlut;
    const int k = T->k;
    std::vector<int16_t> sidx((size_t)k * L.nkeys, -1), xidx((size_t)k * L.nkeys, -1);
    for (int h = 1; h <= k; h++)
        for (int t = 0; t < L.r[h]; t++)
            for (int ci = 0; ci < L.bk[h]; ci++) {
                const uint32_t C = L.mask_k[h][ci];
                const int key = L.off[h] + t * L.bk[h] + ci;
                for (int c = 0; c < k; c++) {
                    const uint32_t D = compress_out(C & ~(1u << c), c);
                    if (C >> c & 1u) {
                        // own count at a colour-c vertex: compressed set of size h-1
                        xidx[(size_t)c * L.nkeys + key] = (int16_t)(t * L.bk1[h - 1] + L.colex_s[D]);
                    } else if (h <= k - 1) {
                        sidx[(size_t)c * L.nkeys + key] = (int16_t)(t * L.bk1[h] + L.colex_s[D]);
                    }
                }
            }
    T->key_sidx = (int16_t *)T->alloc(sidx.size() * 2);
    T->key_xidx = (int16_t *)T->alloc(xidx.size() * 2);
    T->dlut = (DevLut *)T->alloc(sizeof(DevLut));
    if (!T->key_sidx || !T->key_xidx || !T->dlut) return set_error(SCC_ENOMEM, "lookup tables");
    HIP_TRY(hipMemcpyAsync(T->key_sidx, sidx.data(), sidx.size() * 2, hipMemcpyHostToDevice, T->stream));
    HIP_TRY(hipMemcpyAsync(T->key_xidx, xidx.data(), xidx.size() * 2, hipMemcpyHostToDevice, T->stream));
    HIP_TRY(hipMemcpyAsync(T->dlut, &T->hlut, sizeof(DevLut), hipMemcpyHostToDevice, T->stream));
    HIP_TRY(hipStreamSynchronize(T->stream));
    return SCC_OK;
}

extern "C" scc_status scc_build_table(const scc_csr *g, const uint8_t *colors, int k,
                                      const scc_build_opts *opt, scc_table **out)
{
    if (!out) return set_error(SCC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g || !colors) return set_error(SCC_EINVAL, "graph or colours NULL");
    if (k < 2 || k > SCC_KMAX) return set_error(SCC_EINVAL, "k = %d not in [2, 8]", k);
    if (g->n < 0 || g->n >= ((int64_t)1 << 31)) return set_error(SCC_EINVAL, "n out of range");
    if (g->nnz < 0 || (g->n > 0 && (!g->row_ptr || (g->nnz > 0 && !g->col_idx))))
        return set_error(SCC_EINVAL, "bad CSR pointers");
    scc_build_opts o{};
    if (opt) o = *opt;
    if (o.rooting != SCC_ROOT_ZERO && o.rooting != SCC_ROOT_ALL) return set_error(SCC_EINVAL, "bad rooting");
    if (o.max_bits == 0) o.max_bits = 128;
    if (o.max_bits != 64 && o.max_bits != 128) return set_error(SCC_EINVAL, "max_bits must be 64 or 128");

    scc_table *T = new scc_table();
    T->k = k; T->rooting = o.rooting; T->max_bits = o.max_bits;
    T->n = g->n; T->nnz_g = g->nnz;
    T->row_ptr = g->row_ptr; T->col_idx = g->col_idx; T->colors = colors;
    T->stream = (hipStream_t)o.stream;
    T->mem.alloc = o.alloc; T->mem.stream = T->stream;
    build_lut(k, &T->hlut);

    scc_status s = SCC_OK;
    if (o.validate && g->n > 0) {
        int *err = (int *)T->mem.get(16);
        if (!err) { delete T; return set_error(SCC_ENOMEM, "validate"); }
        GraphView gv{g->n, g->row_ptr, g->col_idx, colors};
        int herr = 0;
        hipError_t e = hipMemsetAsync(err, 0, 4, T->stream);
        if (e == hipSuccess) {
            int64_t rp_last = 0;
            e = hipMemcpyAsync(&rp_last, g->row_ptr + g->n, 8, hipMemcpyDeviceToHost, T->stream);
            hipLaunchKernelGGL(k_validate, dim3((unsigned)((g->n + 255) / 256)), dim3(256), 0, T->stream, gv, k, err);
            if (e == hipSuccess) e = hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, T->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(T->stream);
            if (e == hipSuccess && rp_last != g->nnz) herr |= 32;
        }
        T->mem.put(err);
        if (e != hipSuccess) { delete T; return set_error(SCC_EDEVICE, "validate: %s", hipGetErrorString(e)); }
        if (herr) {
            delete T;
            return set_error(SCC_EINVAL, "invalid input (%s%s%s%s%s%s)", herr & 1 ? "colour >= k " : "",
                             herr & 2 ? "row_ptr decreasing " : "", herr & 4 ? "neighbour out of range or self-loop " : "",
                             herr & 8 ? "row not strictly increasing " : "", herr & 16 ? "asymmetric edge " : "",
                             herr & 32 ? "row_ptr[n] != nnz" : "");
        }
    }
    if (!s) s = make_key_maps(T);
    if (!s) s = build_levels(T);
    if (!s) s = build_totals(T);
    if (!s) T->lev[1].nnz = T->n;
    if (s) { delete T; return s; }
    *out = T;
    return SCC_OK;
}

extern "C" void scc_table_destroy(scc_table *t)
{
    if (!t) return;
    (void)hipStreamSynchronize(t->stream);
    delete t;
}

extern "C" scc_status scc_table_info_get(const scc_table *t, scc_table_info *out)
{
    if (!t || !out) return set_error(SCC_EINVAL, "NULL argument");
    memset(out, 0, sizeof *out);
    out->n = t->n; out->k = t->k; out->rooting = t->rooting; out->num_unrooted = t->hlut.num_unr;
    for (int h = 1; h <= t->k; h++) {
        out->nnz[h] = t->lev[h].nnz;
        out->wide_vertices[h] = t->lev[h].wide;
        out->level_ms[h] = t->level_ms[h];
        out->gather_ms[h] = t->gather_ms[h];
        out->gather_bytes[h] = t->gather_bytes[h];
    }
    out->bytes = t->bytes;
    out->t[0] = lo64(t->t); out->t[1] = hi64(t->t);
    for (int j = 0; j < t->hlut.num_unr; j++) { out->tj[j][0] = lo64(t->tj[j]); out->tj[j][1] = hi64(t->tj[j]); }
    return SCC_OK;
}
