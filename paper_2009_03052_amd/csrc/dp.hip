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

#include <map>
#include <mutex>
#include <string>
#include <atomic>
#include <thread>

namespace {


// ---------------------------------------------------------------------------
// CSR and colour validation (Sec. 1.3: simple undirected graph)
// ---------------------------------------------------------------------------
// Pass 1 reads row_ptr only: 0 = row_ptr[0] <= row_ptr[1] <= ... <= row_ptr[n]
// = nnz. Pass 2 runs only when pass 1 found nothing, so its col_idx reads stay
// inside [0, nnz) and its row_ptr reads inside [0, n].
__global__ void k_validate_rows(const int64_t *row_ptr, int64_t n, int64_t nnz, int *err)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > n) return;
    const int64_t a = row_ptr[v];
    int bad = 0;
    if (a < 0 || a > nnz) bad |= 2;
    if (v == 0 && a != 0) bad |= 2;
    if (v == n && a != nnz) bad |= 32;
    if (v < n && row_ptr[v + 1] < a) bad |= 2;
    if (bad) atomicOr(err, bad);
}

// Pass 2, one thread per vertex (its colour) and per CSR entry e: the row v
// holding e, then u = col_idx[e] in range and not v, the row strictly
// increasing at e, and v present in the row of u (symmetry).
__global__ void k_validate_edges(GraphView g, int64_t nnz, int k, int *err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (i < g.n && g.colors[i] >= k) bad |= 1;
    if (i < nnz) {
        int64_t lo = 0, hi = g.n - 1;        // the last v with row_ptr[v] <= i
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (g.row_ptr[mid] <= i) lo = mid; else hi = mid - 1;
        }
        const int64_t v = lo;
        const int32_t u = g.col_idx[i];
        if (u < 0 || u >= g.n || u == v) {
            bad |= 4;
        } else {
            if (i > g.row_ptr[v] && g.col_idx[i - 1] >= u) bad |= 8;
            int64_t a = g.row_ptr[u], b = g.row_ptr[u + 1];
            bool found = false;
            while (a < b) {
                const int64_t mid = (a + b) >> 1;
                const int32_t w = g.col_idx[mid];
                if (w == v) { found = true; break; }
                if (w < v) a = mid + 1; else b = mid;
            }
            if (!found) bad |= 16;
        }
    }
    if (bad) atomicOr(err, bad);
}

// ---------------------------------------------------------------------------
// Level-1 neighbour sums: S_1(v)[j] = number of neighbours of colour j != c_v
// ---------------------------------------------------------------------------
__device__ inline void gather1_vertex(const GraphView &g, int k, uint64_t *S1, u128 *M1, int64_t v, unsigned *cnt)
{
  {
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
    __syncthreads();
  }
}

// Level-1 sums of the vertices v0 + lane (< v1) with at most lane_deg (<= 64)
// neighbours, one vertex per lane: eight 8-bit colour counters packed in one
// word. Returns the ballot of the lanes whose vertex has more neighbours (left
// to the caller).
constexpr int64_t GATHER1_LANE_DEG = 64;
__device__ inline uint64_t gather1_lanes(const GraphView &g, int k, uint64_t *S1, u128 *M1, int64_t v0, int64_t v1,
                                         int64_t lane_deg)
{
    const int64_t v = v0 + lane_id();
    bool big = false;
    if (v < v1) {
        const int64_t a = g.row_ptr[v], b = g.row_ptr[v + 1];
        if (b - a > lane_deg) {
            big = true;
        } else {
            const int cv = g.colors[v];
            uint64_t packed = 0;   // byte c: neighbours of colour c
            int64_t e = a;
            for (; e + 4 <= b; e += 4) {   // four ids, then four colours, in flight together
                int32_t u[4];
#pragma unroll
                for (int j = 0; j < 4; j++) u[j] = g.col_idx[e + j];
#pragma unroll
                for (int j = 0; j < 4; j++) packed += 1ull << (8 * g.colors[u[j]]);
            }
            for (; e < b; e++) packed += 1ull << (8 * g.colors[g.col_idx[e]]);
            for (int c = 0, pos = 0; c < k; c++) {
                if (c == cv) continue;
                S1[v * (k - 1) + pos] = (packed >> (8 * c)) & 0xffu;
                pos++;
            }
            M1[v] = (u128)(b - a);
        }
    }
    return __ballot(big);
}

// one block of 64 vertices per wave (grid-stride), longer rows by the whole
// wave; rows above hub_degree only get zero sums and their degree here, their
// counts coming from k_gather1_hub's chunks
__global__ void __launch_bounds__(WAVE) k_gather1(GraphView g, int k, uint64_t *S1, u128 *M1, int64_t hub_degree)
{
    __shared__ unsigned cnt[SCC_KMAX];
    for (int64_t v0 = (int64_t)blockIdx.x * WAVE; v0 < g.n; v0 += (int64_t)gridDim.x * WAVE) {
        for (uint64_t m = gather1_lanes(g, k, S1, M1, v0, min(g.n, v0 + WAVE), min(GATHER1_LANE_DEG, hub_degree)); m;
             m &= m - 1) {
            const int64_t v = v0 + (__ffsll((long long)m) - 1);
            const int64_t d = g.row_ptr[v + 1] - g.row_ptr[v];
            if (d <= hub_degree) {
                gather1_vertex(g, k, S1, M1, v, cnt);
            } else {
                if (lane_id() < k - 1) S1[v * (k - 1) + lane_id()] = 0;
                if (lane_id() == 0) M1[v] = (u128)d;
            }
        }
    }
}

// level-1 counts of a hub row, one chunk of its neighbours per workgroup, added
// into the row (zeroed by k_gather1, which runs first)
__global__ void __launch_bounds__(WAVE) k_gather1_hub(GraphView g, int k, const int32_t *chunk_v,
                                                      const int64_t *chunk_e, int chunk, uint64_t *S1)
{
    __shared__ unsigned cnt[SCC_KMAX];
    const int lane = threadIdx.x;
    const int64_t v = chunk_v[blockIdx.x];
    const int64_t a = chunk_e[blockIdx.x], b = min(g.row_ptr[v + 1], a + (int64_t)chunk);
    const int cv = g.colors[v];
    if (lane < SCC_KMAX) cnt[lane] = 0;
    __syncthreads();
    for (int64_t e = a + lane; e < b; e += WAVE) {
        const int cu = g.colors[g.col_idx[e]];
        if (cu != cv) atomicAdd(&cnt[cu], 1u);
    }
    __syncthreads();
    if (lane < k && lane != cv && cnt[lane])
        atomicAdd((unsigned long long *)&S1[v * (k - 1) + (lane < cv ? lane : lane - 1)], (unsigned long long)cnt[lane]);
}

// ---------------------------------------------------------------------------
// Gather (the DP join): S_hs(v) = sum over neighbours of their level-hs records,
// plus the bound M_hs(v) = sum_{u~v} N_hs(u) that decides 64- or 128-bit sums.
// Rows of degree <= HUB_DEGREE: one wave per vertex, accumulating in LDS.
// Larger rows: their neighbour list is cut into chunks of HUB_CHUNK, each chunk
// reduced in LDS by one wave and merged into the row with global atomics.
// ---------------------------------------------------------------------------
// Records of one level seen by the gather and the combine: either the packed
// pool (locators + records with a header) or, inside a batched launch, the
// fixed-capacity per-vertex slots the combine writes (meta = len | wide << 31).
// A per-vertex 64-bit handle carries what the accessors need: the locator, or
// (vertex << 32 | meta).
struct LevelSrc {
    LevelView P;
    const uint16_t *skey;
    const uint64_t *slo, *shi;
    const uint32_t *meta;
    const u128 *N;
    int W;
};

template <bool SLOTS> __device__ inline uint64_t src_handle(const LevelSrc &S, int64_t u)
{
    if (SLOTS) return ((uint64_t)u << 32) | S.meta[u];
    return S.P.loc[u];
}
template <bool SLOTS> __device__ inline uint32_t h_len(uint64_t h) { return SLOTS ? META_LEN((uint32_t)h) : LOC_LEN(h); }
template <bool SLOTS> __device__ inline bool h_wide(uint64_t h) { return SLOTS ? META_WIDE((uint32_t)h) != 0 : LOC_WIDE(h) != 0; }
template <bool SLOTS> __device__ inline u128 h_N(const LevelSrc &S, uint64_t h)
{
    if (SLOTS) return h_len<true>(h) ? S.N[h >> 32] : (u128)0;
    if (!LOC_LEN(h)) return 0;
    const uint64_t *p = S.P.pool + LOC_OFF(h);
    return mk128(p[0], p[1]);
}
// keys, low and high words of the entries of the record with handle h
template <bool SLOTS> struct RecView {
    const uint16_t *key;
    const uint64_t *lo, *hi;   // hi is null for a 64-bit record
    uint32_t len;
};
template <bool SLOTS> __device__ inline RecView<SLOTS> h_rec(const LevelSrc &S, uint64_t h)
{
    RecView<SLOTS> r;
    r.len = h_len<SLOTS>(h);
    const bool wide = h_wide<SLOTS>(h);
    if (SLOTS) {
        const size_t base = (size_t)(h >> 32) * S.W;
        r.key = S.skey + base;
        r.lo = S.slo + base;
        r.hi = wide ? S.shi + base : nullptr;
    } else {
        const uint64_t *p = S.P.pool + LOC_OFF(h) + REC_HDR;
        const uint32_t kw = key_words(r.len);
        r.key = (const uint16_t *)p;
        r.lo = p + kw;
        r.hi = wide ? p + kw + r.len : nullptr;
    }
    return r;
}

struct GatherArgs {
    GraphView g;
    int k, nkeys, WS, rows_zero, hub_degree;
    int key_lo, key_n;             // keys of the gathered level: [key_lo, key_lo + key_n), key_n <= GATHER_MAX_KEYS
    LevelSrc L;
    u128 *M;                       // out: M_hs (regular rows); in: hub rows
    const int16_t *key_sidx;       // [k * nkeys]
    uint64_t *Slo, *Shi;           // [n * WS]
    const int32_t *chunk_v;        // hub chunks: vertex and first edge
    const int64_t *chunk_e;
    int *err;
    const DevLut *Lut;             // grouped rows: the level's (rank, colour set) per key
    int hs, bk1;                   // gathered level and binom(k-1, hs)
    // high words in compact rows: hrow[v] = row of v in Shi (hubs first, then the
    // other rows whose bound reaches 2^64, appended to wide_rows by the 64-bit
    // pass); null: Shi has a row for every vertex
    int32_t *hrow;
    int32_t *wide_rows;
    int *wide_count;
    // the sampler's hub running sums built with the gather: each hub chunk (one
    // block of HUB_BLOCK neighbours) stores its sums as its block's (null: not)
    uint64_t *hub_pre;
    const int64_t *hub_poff;       // [nhub * (SCC_KMAX + 1)] word offset of each (hub, level) block area
    const int32_t *chunk_q;        // hub number of each chunk
};

__device__ inline size_t hi_row(const int32_t *hrow, int64_t v) { return hrow ? (size_t)hrow[v] : (size_t)v; }

// most keys on one level: r_6 C(8, 6) = 560 at k = 8
constexpr int GATHER_MAX_KEYS = 576;
// Entries of a chunk of 64 neighbours are spread over the lanes 256 at a time;
// the neighbour owning entry position p is found by marking where every
// neighbour's entries start and taking a running maximum over the positions.
struct OwnerLds {
    uint32_t mark[4 * WAVE];   // 1 + the neighbour lane whose entries start here, or 0
    uint64_t hd[WAVE];         // record handle of each neighbour lane
    uint32_t start[WAVE];      // first entry position of each neighbour lane
    uint32_t tag[WAVE];        // grouped rows: slot | colour << 8 of the lane's row
};

__host__ __device__ inline size_t gather_lds(int WS)
{
    return (size_t)2 * WS * 8 + GATHER_MAX_KEYS * 2 + sizeof(OwnerLds);
}

// owners own[q] of positions q0 + q * WAVE + lane (q = 0..3) among the chunk's
// neighbour lanes, each holding its first position s and entry count len
__device__ inline void round_owners(OwnerLds &O, uint32_t q0, uint32_t s, uint32_t len, int own[4])
{
    const int lane = lane_id();
#pragma unroll
    for (int q = 0; q < 4; q++) O.mark[q * WAVE + lane] = 0;
    __syncthreads();
    if (len && s >= q0 && s < q0 + 4 * WAVE) O.mark[s - q0] = (uint32_t)lane + 1;
    __syncthreads();
    // 1 + the owner of position q0: the last lane with entries starting at or before it
    const uint64_t before = __ballot(len != 0 && s <= q0);
    uint32_t carry = before ? (uint32_t)(WAVE - __clzll((long long)before)) : 0u;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint32_t m = max(wave_incl_max32(O.mark[q * WAVE + lane]), carry);
        carry = (uint32_t)__builtin_amdgcn_readlane((int)m, WAVE - 1);
        own[q] = (int)m - 1;
    }
}

// Adds the level-hs entries of neighbours col_idx[a..b) of v into the LDS sums
// and returns (in every lane) the saturating sum of those neighbours' level
// sums N. With wideS false only low words are added: exact whenever that
// returned bound is below 2^64, since every entry and every partial sum is
// at most the bound. A 64-bit pass stops at the first chunk of neighbours whose
// headers take the bound to 2^64 (the row is redone in 128 bits) and returns
// that partial bound, which is enough to say so.
template <bool SLOTS>
__device__ inline u128 gather_range(const GatherArgs &A, int64_t a, int64_t b, bool wideS, uint64_t *acc_lo,
                                    uint64_t *acc_hi, const int16_t *ssm, OwnerLds &O)
{
    const int lane = threadIdx.x;
    u128 m = 0;
    for (int64_t base = a; base < b; base += WAVE) {
        const int64_t e = base + lane;
        const uint64_t hd = e < b ? src_handle<SLOTS>(A.L, A.g.col_idx[e]) : (SLOTS ? ~0ull << 32 : 0ull);
        const uint32_t len = e < b ? h_len<SLOTS>(hd) : 0u;
        if (len) m = sat_add(m, h_N<SLOTS>(A.L, hd));
        // 64 lane sums below 2^58 each stay below 2^64: the wave sum only when one is not
        if (!wideS && __ballot(hi64(m) != 0 || (lo64(m) >> 58) != 0)) {
            const u128 mt = wave_satsum128(m);
            if (hi64(mt)) return mt;
        }
        const uint32_t incl = wave_incl_scan32(len);
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, WAVE - 1);
        const uint32_t first = incl - len;
        O.hd[lane] = hd;
        O.start[lane] = first;
        // entries of this chunk of neighbours, flattened over the lanes; every lane
        // takes 4 entries per round and issues their loads before using any
        for (uint32_t p0 = 0; p0 < total; p0 += 4 * WAVE) {
            uint32_t key[4];
            uint64_t cl[4], ch[4];
            bool ok[4];
            int own[4];
            round_owners(O, p0, first, len, own);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const uint32_t p = p0 + q * WAVE + lane;
                ok[q] = p < total;
                key[q] = 0;
                cl[q] = ch[q] = 0;
                if (ok[q]) {
                    const RecView<SLOTS> r = h_rec<SLOTS>(A.L, O.hd[own[q]]);
                    const uint32_t ei = p - O.start[own[q]];
                    key[q] = r.key[ei];
                    cl[q] = r.lo[ei];
                    if (wideS && r.hi) ch[q] = r.hi[ei];
                }
            }
#pragma unroll
            for (int q = 0; q < 4; q++) {
                if (!ok[q]) continue;
                const int s = ssm[key[q] - A.key_lo];
                if (s < 0) continue;
                if (!wideS) {
                    atomicAdd((unsigned long long *)&acc_lo[s], (unsigned long long)cl[q]);
                } else {
                    const unsigned long long old = atomicAdd((unsigned long long *)&acc_lo[s], (unsigned long long)cl[q]);
                    const uint64_t carry = (old + cl[q]) < old ? 1u : 0u;
                    if (ch[q] + carry) atomicAdd((unsigned long long *)&acc_hi[s], (unsigned long long)(ch[q] + carry));
                }
            }
        }
        __syncthreads();   // the next chunk rewrites the lane table
    }
    return wave_satsum128(m);
}

// LDS sums of the neighbours in [a, b): 64-bit pass first, a 128-bit pass only
// when the bound says 64 bits may not suffice
// LDS: acc_lo[WS], acc_hi[WS], then the index slice of colour cv (GATHER_MAX_KEYS int16)
// mode: GS_BOTH (64-bit pass, then 128-bit if the bound needs it), GS_DEFER
// (64-bit pass only; wideS reports the need), GS_WIDE (128-bit pass only)
enum { GS_BOTH = 0, GS_DEFER = 1, GS_WIDE = 2 };
template <bool SLOTS>
__device__ inline u128 gather_sums(const GatherArgs &A, int cv, int64_t a, int64_t b, uint64_t *acc_lo,
                                   uint64_t *acc_hi, bool &wideS, int mode = GS_BOTH)
{
    const int lane = threadIdx.x;
    const int WS = A.WS;
    int16_t *ssm = (int16_t *)(acc_hi + WS);
    OwnerLds &O = *(OwnerLds *)(ssm + GATHER_MAX_KEYS);
    const int16_t *sidx = A.key_sidx + (size_t)cv * A.nkeys + A.key_lo;
    for (int i = lane; i < A.key_n; i += WAVE) ssm[i] = sidx[i];
    for (int i = lane; i < WS; i += WAVE) { acc_lo[i] = 0; acc_hi[i] = 0; }
    __syncthreads();
    u128 m = 0;
    wideS = mode == GS_WIDE;
    if (!wideS) {
        m = gather_range<SLOTS>(A, a, b, false, acc_lo, acc_hi, ssm, O);
        wideS = hi64(m) != 0;
    }
    if (wideS && mode != GS_DEFER) {
        __syncthreads();
        for (int i = lane; i < WS; i += WAVE) { acc_lo[i] = 0; acc_hi[i] = 0; }
        __syncthreads();
        m = gather_range<SLOTS>(A, a, b, true, acc_lo, acc_hi, ssm, O);
    }
    __syncthreads();
    return m;
}

// GS_DEFER: a row whose bound reaches 2^64 is only listed (its 128-bit pass
// runs, GS_WIDE, once its compact high-word row exists)
template <bool SLOTS>
__device__ inline void gather_vertex(const GatherArgs &A, int64_t v, uint64_t *sm, int mode = GS_BOTH)
{
    const int lane = threadIdx.x;
    const int cv = A.g.colors[v];
    if (A.rows_zero && cv != 0) return;
    const int64_t a = A.g.row_ptr[v], b = A.g.row_ptr[v + 1];
    if (b - a > A.hub_degree) return;      // hub rows have their own kernels
    const int WS = A.WS;
    uint64_t *acc_lo = sm;
    uint64_t *acc_hi = sm + WS;
    bool wideS;
    // bound: every entry of S_hs(v) is at most M_hs(v)
    const u128 m = gather_sums<SLOTS>(A, cv, a, b, acc_lo, acc_hi, wideS, mode);
    if (wideS && mode == GS_DEFER) {
        if (lane == 0) A.wide_rows[atomicAdd(A.wide_count, 1)] = (int32_t)v;
        return;
    }
    uint64_t *Slo = A.Slo + (size_t)v * WS;
    for (int i = lane; i < WS; i += WAVE) Slo[i] = acc_lo[i];
    if (wideS) {
        uint64_t *Shi = A.Shi + hi_row(A.hrow, v) * WS;
        for (int i = lane; i < WS; i += WAVE) Shi[i] = acc_hi[i];
    }
    if (lane == 0) A.M[v] = m;
}

// one row per wave, every row below the hub threshold
__global__ void __launch_bounds__(WAVE) k_gather(GatherArgs A)
{
    extern __shared__ uint64_t sm[];
    for (int64_t v = blockIdx.x; v < A.g.n; v += gridDim.x) {
        gather_vertex<false>(A, v, sm, A.hrow ? GS_DEFER : GS_BOTH);
        __syncthreads();
    }
}

// rows from a list (the rows between the grouped ones and the hubs)
__global__ void __launch_bounds__(WAVE) k_gather_list(GatherArgs A, const int32_t *rows)
{
    extern __shared__ uint64_t sm[];
    gather_vertex<false>(A, rows[blockIdx.x], sm, A.hrow ? GS_DEFER : GS_BOTH);
}

// the listed rows whose bound reaches 2^64 (one per workgroup), 128-bit pass
// into their compact high-word rows
__global__ void __launch_bounds__(WAVE) k_gather_wide(GatherArgs A)
{
    extern __shared__ uint64_t sm[];
    gather_vertex<false>(A, __builtin_amdgcn_readfirstlane(A.wide_rows[blockIdx.x]), sm, GS_WIDE);
}

// Which rows of a level's gather need 128-bit sums, one row per lane: the
// bound M_hs(v), the saturating sum of the neighbours' level sums N (read from
// the combine's per-vertex array N, equal to the records' headers) as the
// 64-bit pass forms it. Rows whose bound reaches 2^64 go to wide_rows, as that
// pass would list them; the others to narrow (*ncount) for it; hub rows are
// left to their kernels. Used where many rows are wide: the 64-bit pass would
// start each of them only to stop. (A lane per row measured faster than 2, 4,
// 8, 16 or 64 lanes per row: 101, 102, 105, 110, 117 and 145 ms for the large
// workload's level-6 sums.)
__global__ void __launch_bounds__(256) k_gather_classify(GatherArgs A, const u128 *N, int32_t *narrow, int *ncount)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = v < A.g.n;
    const int64_t a = in ? A.g.row_ptr[v] : 0, b = in ? A.g.row_ptr[v + 1] : 0;
    const bool act = in && b - a <= A.hub_degree;
    u128 m = 0;
    // four neighbours at a time, their loads issued before any is summed
    for (int64_t e0 = a; act && e0 < b; e0 += 4) {
        int32_t u[4];
        u128 x[4];
#pragma unroll
        for (int j = 0; j < 4; j++) u[j] = e0 + j < b ? A.g.col_idx[e0 + j] : -1;
#pragma unroll
        for (int j = 0; j < 4; j++) x[j] = u[j] >= 0 ? N[u[j]] : (u128)0;
#pragma unroll
        for (int j = 0; j < 4; j++) m = sat_add(m, x[j]);
    }
    const bool wide = act && hi64(m) != 0, nar = act && !wide;
    const uint64_t bw = __ballot(wide), bn = __ballot(nar);
    int bw0 = 0, bn0 = 0;
    if (lane_id() == 0) {
        if (bw) bw0 = atomicAdd(A.wide_count, __popcll(bw));
        if (bn) bn0 = atomicAdd(ncount, __popcll(bn));
    }
    bw0 = __shfl(bw0, 0);
    bn0 = __shfl(bn0, 0);
    const uint64_t below = lanemask_lt();
    if (wide) A.wide_rows[bw0 + __popcll(bw & below)] = (int32_t)v;
    if (nar) narrow[bn0 + __popcll(bn & below)] = (int32_t)v;
}

// the degrees of the vertices whose level sum N has a high word, summed: the
// rows of the next level's gather that will need 128-bit sums are at least
// their neighbours
__global__ void __launch_bounds__(256) k_heavy_degree(GraphView g, const u128 *N, unsigned long long *out)
{
    unsigned long long d = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += (int64_t)gridDim.x * blockDim.x)
        if (hi64(N[v])) d += (unsigned long long)(g.row_ptr[v + 1] - g.row_ptr[v]);
    d = wave_sum64(d);
    if (lane_id() == 0 && d) atomicAdd(out, d);
}

// hrow[rows[i]] = base + i
__global__ void k_set_rows(int32_t *hrow, const int32_t *rows, const int *count, int64_t fixed, int32_t base)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cnt = count ? (int64_t)*count : fixed;
    if (i < cnt) hrow[rows[i]] = base + (int32_t)i;
}

// ---------------------------------------------------------------------------
// Low-degree rows in groups: one wave gathers G consecutive vertices of degree
// at most GROUP_DEG (and not above the hub threshold), so that the neighbours
// and record entries of several rows fill the lanes; most rows of a
// heavy-tailed graph have a handful of neighbours. The sums of the group's
// rows accumulate in G rows of LDS; the slot of a key at a colour-c vertex is
// rank(T'') binom(k-1, hs) + colex of C'' without c, from a per-level table of
// (rank, colour set) and the colex table, shared by every colour.
// ---------------------------------------------------------------------------
constexpr int GROUP_DEG = 64;
constexpr int GROUP_MAX = 8;
// SCC_GATHER_AUTO groups a level when at least half the rows have at most
// GROUP_LOW_DEG neighbours and the level's records average at most GROUP_WORDS
// pool words (about 32 entries): then a wave per row leaves most lanes idle
constexpr int GROUP_LOW_DEG = 8;
constexpr int GROUP_WORDS = 40;

inline int group_size(int WS) { return std::max(2, std::min(GROUP_MAX, 512 / std::max(1, WS))); }
inline size_t group_lds(int WS, int G)
{
    return (size_t)G * WS * 8 + (gather_lds(WS) + 7) / 8 * 8 + GATHER_MAX_KEYS * 2 + 128;
}

template <bool SLOTS>
__device__ inline void gather_group(const GatherArgs &A, int64_t v0, int G, uint64_t *acc, const uint16_t *kinfo,
                                    const uint8_t *colex, uint64_t *wsm)
{
    const int lane = threadIdx.x;
    const int WS = A.WS;
    const int nv = (int)min((int64_t)G, A.g.n - v0);
    const int64_t small = min((int64_t)GROUP_DEG, (int64_t)A.hub_degree);
    // lane j < nv describes vertex v0 + j
    int64_t ra = 0;
    uint32_t dj = 0;
    int cvj = 0;
    bool mine = false;
    if (lane < nv) {
        const int64_t v = v0 + lane;
        ra = A.g.row_ptr[v];
        const int64_t d = A.g.row_ptr[v + 1] - ra;
        cvj = A.g.colors[v];
        mine = d <= small && !(A.rows_zero && cvj != 0);
        dj = mine ? (uint32_t)d : 0u;
    }
    const uint64_t mine_mask = __ballot(mine);
    if (!mine_mask) return;
    OwnerLds &O = *(OwnerLds *)((int16_t *)(wsm + 2 * WS) + GATHER_MAX_KEYS);
    const uint32_t dincl = wave_incl_scan32(dj);
    const uint32_t E = __shfl(dincl, WAVE - 1, WAVE);
    for (int i = lane; i < nv * WS; i += WAVE) acc[i] = 0;
    __syncthreads();
    u128 mj = 0;   // lane j < nv: bound of vertex v0 + j (sum of its neighbours' level sums)
    for (uint32_t p0 = 0; p0 < E; p0 += WAVE) {
        const uint32_t p = p0 + lane;
        // slot of edge position p: the number of slots whose inclusive degree is <= p
        int js = 0;
#pragma unroll
        for (int step = GROUP_MAX / 2; step >= 1; step >>= 1) {
            const uint32_t x = __shfl(dincl, js + step - 1, WAVE);
            if (x <= p) js += step;
        }
        const uint32_t dincl_s = __shfl(dincl, js, WAVE);
        const uint32_t d_s = __shfl(dj, js, WAVE);
        const int64_t ra_s = (int64_t)shfl64((uint64_t)ra, js);
        uint64_t hd = SLOTS ? ~0ull << 32 : 0ull;
        uint32_t len = 0;
        u128 nval = 0;
        if (p < E) {
            hd = src_handle<SLOTS>(A.L, A.g.col_idx[ra_s + (int64_t)(p - (dincl_s - d_s))]);
            len = h_len<SLOTS>(hd);
            if (len) nval = h_N<SLOTS>(A.L, hd);
        }
        // each slot's lanes are contiguous: its bound grows by their segment of the scan
        const u128 incl_n = wave_incl_satscan128(nval);
        const int sa = (int)max(dincl - dj, p0) - (int)p0;
        const int sb = (int)min(dincl, p0 + WAVE) - (int)p0;
        const u128 before = shfl128(incl_n, max(sa - 1, 0));
        const u128 last = shfl128(incl_n, max(sb - 1, 0));
        if (lane < nv && sb > sa) {
            const u128 seg = last == ~(u128)0 ? ~(u128)0 : last - (sa > 0 ? before : (u128)0);
            mj = sat_add(mj, seg);
        }
        // the entries of these neighbours, flattened, 4 per lane per round
        const uint32_t incl = wave_incl_scan32(len);
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, WAVE - 1);
        const uint32_t first = incl - len;
        const int cv_s = __shfl(cvj, js, WAVE);
        O.hd[lane] = hd;
        O.start[lane] = first;
        O.tag[lane] = (uint32_t)js | ((uint32_t)cv_s << 8);
        for (uint32_t q0 = 0; q0 < total; q0 += 4 * WAVE) {
            uint32_t key[4];
            uint64_t cl[4];
            int slot[4], cv[4];
            bool ok[4];
            int own[4];
            round_owners(O, q0, first, len, own);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const uint32_t pe = q0 + q * WAVE + lane;
                ok[q] = pe < total;
                key[q] = 0;
                cl[q] = 0;
                slot[q] = cv[q] = 0;
                if (ok[q]) {
                    const uint32_t tag = O.tag[own[q]];
                    slot[q] = (int)(tag & 0xffu);
                    cv[q] = (int)(tag >> 8);
                    const RecView<SLOTS> r = h_rec<SLOTS>(A.L, O.hd[own[q]]);
                    const uint32_t ei = pe - O.start[own[q]];
                    key[q] = r.key[ei];
                    cl[q] = r.lo[ei];
                }
            }
#pragma unroll
            for (int q = 0; q < 4; q++) {
                if (!ok[q]) continue;
                const uint32_t km = kinfo[key[q] - A.key_lo];
                const uint32_t C = km & 0xffu;
                if (C >> cv[q] & 1u) continue;   // a colour set holding c_v is not summed
                const int s = (int)(km >> 8) * A.bk1 + colex[compress_out(C, cv[q])];
                atomicAdd((unsigned long long *)&acc[slot[q] * WS + s], (unsigned long long)cl[q]);
            }
        }
        __syncthreads();   // the next chunk rewrites the lane table
    }
    __syncthreads();
    // rows whose bound reaches 2^64 are redone alone with 128-bit sums
    const uint64_t wide_mask = __ballot(lane < nv && mine && hi64(mj) != 0);
    uint64_t *Slo = A.Slo + (size_t)v0 * WS;
    for (int i = lane; i < nv * WS; i += WAVE) {
        const int j = i / WS;
        if ((mine_mask >> j & 1u) && !(wide_mask >> j & 1u)) Slo[i] = acc[i];
    }
    if (lane < nv && mine && !(wide_mask >> lane & 1u)) A.M[v0 + lane] = mj;
    if (A.hrow) {
        // listed for the 128-bit pass once their high-word rows exist
        const int nw = __popcll(wide_mask);
        int base = 0;
        if (nw && lane == 0) base = atomicAdd(A.wide_count, nw);
        base = __shfl(base, 0, WAVE);
        if (wide_mask >> lane & 1u) A.wide_rows[base + __popcll(wide_mask & lanemask_lt())] = (int32_t)(v0 + lane);
    } else {
        for (uint64_t wm = wide_mask; wm; wm &= wm - 1) {
            __syncthreads();
            gather_vertex<SLOTS>(A, v0 + (__ffsll((long long)wm) - 1), wsm);
        }
    }
}

// LDS: G * WS sums, the single-row area for 128-bit rows, the key table, the colex table
__global__ void __launch_bounds__(WAVE) k_gather_group(GatherArgs A, int G)
{
    extern __shared__ uint64_t sm[];
    const int WS = A.WS;
    uint64_t *acc = sm;
    uint64_t *wsm = acc + (size_t)G * WS;
    uint16_t *kinfo = (uint16_t *)(wsm + (gather_lds(WS) + 7) / 8);
    uint8_t *colex = (uint8_t *)(kinfo + GATHER_MAX_KEYS);
    const DevLut &L = *A.Lut;
    const int bk = L.bk[A.hs];
    for (int i = threadIdx.x; i < A.key_n; i += WAVE) {
        const int t = i / bk;
        kinfo[i] = (uint16_t)((t << 8) | L.mask_k[A.hs][i - t * bk]);
    }
    for (int i = threadIdx.x; i < 128; i += WAVE) colex[i] = L.colex_s[i];
    __syncthreads();
    const int64_t ng = (A.g.n + G - 1) / G;
    for (int64_t gi = blockIdx.x; gi < ng; gi += gridDim.x) {
        gather_group<false>(A, gi * G, G, acc, kinfo, colex, wsm);
        __syncthreads();
    }
}

// hub rows, step 1: cleared sums and bound
__device__ inline void hub_zero(const GatherArgs &A, int64_t v)
{
    const size_t hr = hi_row(A.hrow, v);
    for (int i = threadIdx.x; i < A.WS; i += blockDim.x) {
        A.Slo[(size_t)v * A.WS + i] = 0;
        A.Shi[hr * A.WS + i] = 0;
    }
    if (threadIdx.x == 0) A.M[v] = 0;
}

__global__ void __launch_bounds__(WAVE) k_hub_prepare(GatherArgs A, const int32_t *hubs)
{
    hub_zero(A, hubs[blockIdx.x]);
}

// adds a 128-bit value to a 128-bit word pair with device atomics; returns
// true when the sum leaves 128 bits
__device__ inline bool atomic_add128(unsigned long long *lo_w, unsigned long long *hi_w, uint64_t lo, uint64_t hi)
{
    const unsigned long long old = atomicAdd(lo_w, (unsigned long long)lo);
    const uint64_t carry = (old + lo) < old ? 1u : 0u;
    const uint64_t add = hi + carry;
    if (add == 0 && !(hi != 0 && carry)) return false;
    const unsigned long long oldh = atomicAdd(hi_w, (unsigned long long)add);
    return (oldh + add) < oldh || (carry && hi == ~0ull);
}

// hub rows, step 2: one wave per chunk of neighbours, merged with atomics
template <bool SLOTS>
__device__ inline void hub_chunk(const GatherArgs &A, int64_t v, int64_t a, int64_t b, uint64_t *sm, int q = -1)
{
    const int lane = threadIdx.x;
    const int cv = A.g.colors[v];
    const int WS = A.WS;
    uint64_t *acc_lo = sm;
    uint64_t *acc_hi = sm + WS;
    bool wideS;
    const u128 m = gather_sums<SLOTS>(A, cv, a, b, acc_lo, acc_hi, wideS);
    unsigned long long *Slo = (unsigned long long *)(A.Slo + (size_t)v * WS);
    unsigned long long *Shi = (unsigned long long *)(A.Shi + hi_row(A.hrow, v) * WS);
    bool over = false;
    for (int i = lane; i < WS; i += WAVE) {
        const uint64_t lo = acc_lo[i], hi = acc_hi[i];
        if (lo || hi) over |= atomic_add128(&Slo[i], &Shi[i], lo, hi);
    }
    if (lane == 0) {
        unsigned long long *Mw = (unsigned long long *)&A.M[v];
        over |= atomic_add128(&Mw[0], &Mw[1], lo64(m), hi64(m));
        if (m == ~(u128)0) over = true;
    }
    if (over) atomicOr(A.err, 2);   // the bound left 128 bits: the build reports overflow
    if (A.hub_pre && q >= 0 && !(A.rows_zero && cv != 0)) {
        // this chunk is block (a - row start) / HUB_BLOCK of the hub's running sums
        const int64_t ra = A.g.row_ptr[v], d = A.g.row_ptr[v + 1] - ra;
        const int64_t nb = (d + HUB_BLOCK - 1) / HUB_BLOCK, blk = (a - ra) / HUB_BLOCK;
        uint64_t *plo = A.hub_pre + A.hub_poff[(size_t)q * (SCC_KMAX + 1) + A.hs];
        uint64_t *phi = plo + (size_t)WS * nb;
        for (int i = lane; i < WS; i += WAVE) {
            plo[(size_t)i * nb + blk] = acc_lo[i];
            phi[(size_t)i * nb + blk] = acc_hi[i];
        }
    }
}

// level-1 block sums of the hub running sums: neighbours of each colour per block
__global__ void __launch_bounds__(WAVE) k_hub_l1_blocks(GraphView g, int k, const int32_t *hubs,
                                                        const int64_t *chunk_e, const int32_t *chunk_q,
                                                        uint64_t *hub_pre, const int64_t *hub_poff)
{
    const int lane = threadIdx.x;
    const int q = chunk_q[blockIdx.x];
    const int64_t x = hubs[q];
    const int cx = g.colors[x];
    const int64_t ra = g.row_ptr[x], rb = g.row_ptr[x + 1], a = chunk_e[blockIdx.x];
    const int64_t nb = (rb - ra + HUB_BLOCK - 1) / HUB_BLOCK, blk = (a - ra) / HUB_BLOCK;
    const int64_t e = a + lane;
    int j = -1;
    if (e < rb && lane < HUB_BLOCK) {
        const int cu = g.colors[g.col_idx[e]];
        if (cu != cx) j = cu < cx ? cu : cu - 1;   // the S_1 entry of colour set {c_u} seen from x
    }
    uint64_t *plo = hub_pre + hub_poff[(size_t)q * (SCC_KMAX + 1) + 1];
    uint64_t *phi = plo + (size_t)(k - 1) * nb;
    for (int i = 0; i < k - 1; i++) {
        const uint64_t c = (uint64_t)__popcll(__ballot(j == i));
        if (lane == 0) {
            plo[(size_t)i * nb + blk] = c;
            phi[(size_t)i * nb + blk] = 0;
        }
    }
}

// block sums -> running sums at block ends, in place: one wave per (hub, entry),
// 64 blocks per step; high words kept only where the hub's bound M reaches 2^64
__global__ void __launch_bounds__(WAVE) k_hub_block_scan(GraphView g, const int32_t *hubs, int WS, int hs,
                                                         int rows_zero, const u128 *M, uint64_t *hub_pre,
                                                         const int64_t *hub_poff)
{
    const int q = blockIdx.x / WS, i = blockIdx.x - q * WS;
    const int64_t x = hubs[q];
    if (rows_zero && g.colors[x] != 0) return;
    const int64_t nb = (g.row_ptr[x + 1] - g.row_ptr[x] + HUB_BLOCK - 1) / HUB_BLOCK;
    uint64_t *plo = hub_pre + hub_poff[(size_t)q * (SCC_KMAX + 1) + hs];
    uint64_t *phi = plo + (size_t)WS * nb;
    plo += (size_t)i * nb;
    phi += (size_t)i * nb;
    const bool pw = hi64(M[x]) != 0;
    u128 carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += WAVE) {
        const int64_t b = b0 + threadIdx.x;
        const u128 val = b < nb ? mk128(plo[b], phi[b]) : (u128)0;
        const u128 run = carry + wave_incl_scan128(val);
        if (b < nb) {
            plo[b] = lo64(run);
            if (pw) phi[b] = hi64(run);
        }
        carry = shfl128(run, WAVE - 1);
    }
}

__global__ void __launch_bounds__(WAVE) k_gather_hub(GatherArgs A, int chunk)
{
    extern __shared__ uint64_t sm[];
    const int64_t v = A.chunk_v[blockIdx.x];
    const int64_t a = A.chunk_e[blockIdx.x];
    const int64_t b = min(A.g.row_ptr[v + 1], a + (int64_t)chunk);
    hub_chunk<false>(A, v, a, b, sm, A.chunk_q ? A.chunk_q[blockIdx.x] : -1);
}

// algorithmic bytes of one gather launch (for reports): 4 d_v + neighbours'
// records (10 B per 64-bit entry, 18 B per 128-bit entry) + the sums written
__global__ void __launch_bounds__(256) k_gather_bytes(GraphView g, LevelView L, const u128 *M, int WS, int rows_zero,
                                                      unsigned long long *out)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t bytes = 0;
    if (v < g.n && (!rows_zero || g.colors[v] == 0)) {
        const int64_t a = g.row_ptr[v], b = g.row_ptr[v + 1];
        bytes = 4ull * (uint64_t)(b - a) + (uint64_t)WS * (hi64(M[v]) ? 16u : 8u);
        for (int64_t e = a; e < b; e++) {
            const uint64_t l = L.loc[g.col_idx[e]];
            bytes += (uint64_t)LOC_LEN(l) * (LOC_WIDE(l) ? 18u : 10u);
        }
    }
    bytes = wave_sum64(bytes);
    if (lane_id() == 0 && bytes) atomicAdd(out, (unsigned long long)bytes);
}

// Algorithmic bytes of the combine of every level h >= 2 at each vertex that
// has level h (under zero-rooting level k only at colour-0 vertices): Eq. (1)
// reads the vertex's own records of levels 2..h-1 (10 B per entry, 18 B for a
// 128-bit vertex; level 1 is implicit) and its dense neighbour sums of levels
// 1..h-1 that exist (8 B per entry, 16 B for rows with high words), and writes
// its level-h record. out[h] accumulates level h; out[0] the level-k totals
// (the level-k records read, eta and its running sum written: 32 B a vertex).
struct CombineBytesArgs {
    GraphView g;
    int k, zero;
    LevelView lev[SCC_KMAX + 1];
    const int32_t *hrow[SCC_KMAX + 1];
    int WS[SCC_KMAX + 1];
    int s_built[SCC_KMAX + 1];
};

__global__ void __launch_bounds__(256) k_combine_bytes(CombineBytesArgs A, unsigned long long *out)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t own[SCC_KMAX + 1] = {0}, sums[SCC_KMAX + 1] = {0};
    uint64_t by[SCC_KMAX + 1] = {0};
    if (v < A.g.n) {
        for (int h = 2; h <= A.k; h++) {
            const uint64_t l = A.lev[h].loc[v];
            own[h] = (uint64_t)LOC_LEN(l) * (LOC_WIDE(l) ? 18u : 10u);
        }
        for (int h = 1; h < A.k; h++)
            if (A.s_built[h]) sums[h] = (uint64_t)A.WS[h] * ((h >= 2 && A.hrow[h] && A.hrow[h][v] >= 0) ? 16u : 8u);
        uint64_t below = sums[1];
        for (int h = 2; h <= A.k; h++) {
            const bool here = !(A.zero && h == A.k && A.g.colors[v] != 0);
            if (here) by[h] = below + own[h];
            below += own[h] + sums[h];
        }
        by[0] = own[A.k] + 32u;
    }
    for (int h = 0; h <= A.k; h++) {
        if (h == 1) continue;
        const uint64_t b = wave_sum64(by[h]);
        if (lane_id() == 0 && b) atomicAdd(out + h, (unsigned long long)b);
    }
}

__global__ void k_hub_rows(GraphView g, const int32_t *hubs, int nhub, int64_t *rows)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nhub) return;
    rows[2 * i] = g.row_ptr[hubs[i]];
    rows[2 * i + 1] = g.row_ptr[hubs[i] + 1];
}

__global__ void k_hub_list(GraphView g, int hub_degree, int32_t *hubs, int *count)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    if (g.row_ptr[v + 1] - g.row_ptr[v] > hub_degree) hubs[atomicAdd(count, 1)] = (int32_t)v;
}

// hub rows (count[0]), the rows between the grouped ones and the hubs
// (count[1]), the number of rows of at most GROUP_LOW_DEG neighbours (count[2])
// and the colour-0 rows (count[3]), each list in no particular order. One atomic
// per list and block of ROW_LIST_T rows: the four counters are shared by the
// whole grid.
constexpr int ROW_LIST_T = 1024;
__global__ void __launch_bounds__(ROW_LIST_T) k_row_lists(GraphView g, int hub_degree, int32_t *hubs, int32_t *mids,
                                                           int32_t *zrows, int *count)
{
    __shared__ int wcnt[ROW_LIST_T / WAVE][4];   // per wave: hubs, mids, colour-0 rows, low rows
    __shared__ int wbase[ROW_LIST_T / WAVE][3];
    const int w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t d = v < g.n ? g.row_ptr[v + 1] - g.row_ptr[v] : 0;
    const bool hub = v < g.n && d > hub_degree, mid = v < g.n && !hub && d > GROUP_DEG;
    const bool zero = v < g.n && g.colors[v] == 0;
    const uint64_t hm = __ballot(hub), mm = __ballot(mid), zm = __ballot(zero);
    const uint64_t low = __ballot(v < g.n && d <= GROUP_LOW_DEG);
    if (lane_id() == 0) {
        wcnt[w][0] = __popcll(hm);
        wcnt[w][1] = __popcll(mm);
        wcnt[w][2] = __popcll(zm);
        wcnt[w][3] = __popcll(low);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot[4] = {0, 0, 0, 0};
        for (int q = 0; q < nw; q++)
            for (int l = 0; l < 3; l++) {
                wbase[q][l] = tot[l];
                tot[l] += wcnt[q][l];
            }
        for (int q = 0; q < nw; q++) tot[3] += wcnt[q][3];
        const int b0 = tot[0] ? atomicAdd(&count[0], tot[0]) : 0;
        const int b1 = tot[1] ? atomicAdd(&count[1], tot[1]) : 0;
        const int b2 = tot[2] ? atomicAdd(&count[3], tot[2]) : 0;
        if (tot[3]) atomicAdd(&count[2], tot[3]);
        for (int q = 0; q < nw; q++) {
            wbase[q][0] += b0;
            wbase[q][1] += b1;
            wbase[q][2] += b2;
        }
    }
    __syncthreads();
    if (hub) hubs[wbase[w][0] + __popcll(hm & lanemask_lt())] = (int32_t)v;
    if (mid) mids[wbase[w][1] + __popcll(mm & lanemask_lt())] = (int32_t)v;
    if (zero) zrows[wbase[w][2] + __popcll(zm & lanemask_lt())] = (int32_t)v;
}

// ---------------------------------------------------------------------------
// Combine: Eq. (1) with the neighbour sum already formed
// ---------------------------------------------------------------------------
struct CombineArgs {
    GraphView g;
    const DevLut *L;
    int h, zero_only, max_bits;
    int bal;                              // level k under round skipping: designated shapes only
    LevelSrc lev[SCC_KMAX + 1];           // own levels 2..h-1
    const uint64_t *Slo[SCC_KMAX + 1];    // neighbour sums 1..h-1
    const uint64_t *Shi[SCC_KMAX + 1];
    const int32_t *Shrow[SCC_KMAX + 1];   // compact high-word rows, or null (one per vertex)
    const u128 *M[SCC_KMAX + 1];
    const int16_t *key_xidx;              // [k * nkeys]
    int W;                                // slot capacity = W_h
    int late_dma;                         // listing passes stage the sums after the width test
    int hi_cap;                           // > 0: words of LDS for staged sum high words (checked)
    uint16_t *slot_key;
    uint64_t *slot_lo, *slot_hi;          // slot_hi may be null (no wide vertex)
    uint32_t *meta;
    u128 *Nout;
    int *err;                             // [0]: overflow
    uint64_t *bm;                         // the level's presence bitmaps (BW words a vertex), or null
    int BW;
};

template <int ILP>
__device__ inline void combine_outputs(const CombineArgs &A, int64_t v, int cv, const uint64_t *Xlo,
                                       const uint64_t *Slo, const uint64_t *Xhi, const uint64_t *Shi, bool owide,
                                       bool wide, int s_hi0 = 0, const uint16_t *tx_lds = nullptr);

// Counts of vertex v at level h. The low words of v's own counts X and of its
// neighbour sums S are staged in lo_area (LDS); high words are needed only when
// v's bound U reaches 2^64 and are staged in hi_area. With hi_area null, such a
// vertex is appended to wide_list instead and left for a second pass.
template <bool SLOTS>
__device__ inline void combine_vertex(const CombineArgs &A, int64_t v, uint64_t *lo_area, uint64_t *hi_area,
                                      int *wide_list, int *wide_count)
{
    const DevLut &L = *A.L;
    const int lane = threadIdx.x;
    const int h = A.h;
    const int cv = A.g.colors[v];
    if (A.zero_only && cv != 0) {
        if (lane == 0) { A.meta[v] = 0; A.Nout[v] = 0; }
        return;
    }
    // per-vertex bound: U >= sum over (T, C) of beta_T c(T_C, v) >= every partial sum.
    // Under round skipping both parts of a designated shape have 2..h-2 nodes, so
    // only those part sizes are bounded and staged (level h-1 is not built).
    const int plo = A.bal ? 2 : 1, phi = A.bal ? h - 2 : h - 1;
    u128 U = 0;
    for (int hp = plo; hp <= phi; hp++) {
        if (!A.M[h - hp]) continue;   // sums not built: no evaluated term uses them
        u128 Nv = hp == 1 ? (u128)1 : h_N<SLOTS>(A.lev[hp], src_handle<SLOTS>(A.lev[hp], v));
        U = sat_add(U, sat_mul(Nv, A.M[h - hp][v]));
    }
    if (U == ~(u128)0 || bitlen128(U) > A.max_bits) {
        if (lane == 0) { atomicOr(A.err, 1); A.meta[v] = 0; A.Nout[v] = 0; }
        return;
    }
    // owide: some output or partial sum may reach 2^64 (accumulate and store 128
    // bits); wide: some input has high words too (stage them). Below 2^64 every
    // product and partial sum fits in the low words (U bounds them).
    const bool owide = hi64(U) != 0;
    bool wide = false;
    if (owide) {
        for (int hp = 2; hp <= phi; hp++) wide |= h_wide<SLOTS>(src_handle<SLOTS>(A.lev[hp], v));
        for (int hs = 1; hs <= phi; hs++) wide |= A.M[hs] && hi64(A.M[hs][v]) != 0;
    }
    if (wide && !hi_area) {
        if (lane == 0) wide_list[atomicAdd(wide_count, 1)] = (int)v;
        return;
    }
    const int XT = L.xoff[h];
    uint64_t *Xlo = lo_area, *Slo = lo_area + XT;
    uint64_t *Xhi = hi_area, *Shi = hi_area + XT;
    for (int i = lane; i < XT; i += WAVE) {
        Xlo[i] = 0;
        if (wide) Xhi[i] = 0;
    }
    __syncthreads();
    if (lane == 0) Xlo[L.xoff[1]] = 1;   // level 1: the single node, coloured c_v
    const int16_t *xidx = A.key_xidx + (size_t)cv * L.nkeys;
    for (int hp = 2; hp <= phi; hp++) {
        const RecView<SLOTS> r = h_rec<SLOTS>(A.lev[hp], src_handle<SLOTS>(A.lev[hp], v));
        for (uint32_t e = lane; e < r.len; e += WAVE) {
            const int x = L.xoff[hp] + xidx[r.key[e]];
            Xlo[x] = r.lo[e];
            if (wide) Xhi[x] = r.hi ? r.hi[e] : 0;
        }
    }
    for (int hs = 1; hs <= phi; hs++) {
        if (!A.Slo[hs]) continue;
        const int ws = L.WS[hs];
        const uint64_t *gl = A.Slo[hs] + (size_t)v * ws;
        const bool sw = hi64(A.M[hs][v]) != 0;
        const uint64_t *gh = sw ? A.Shi[hs] + hi_row(A.Shrow[hs], v) * ws : nullptr;
        for (int i = lane; i < ws; i += WAVE) {
            Slo[L.soff[hs] + i] = gl[i];
            if (wide) Shi[L.soff[hs] + i] = sw ? gh[i] : 0;
        }
    }
    __syncthreads();
    combine_outputs<4>(A, v, cv, Xlo, Slo, Xhi, Shi, owide, wide);
}

// The outputs of vertex v at level h from its staged counts (X) and neighbour
// sums (S): lane o evaluates outputs o, o + 64, ..., and the nonzero ones are
// compacted into v's slot right away (ballot + prefix count keeps ascending
// key order).
// x s modulo 2^128 (the vertex's bound keeps every product below it)
__device__ inline u128 mul_64x128(uint64_t x, u128 s) { return (u128)x * lo64(s) + ((u128)(x * hi64(s)) << 64); }

// ILP = 4: an output's terms four at a time (the level kernels); ILP = 1: one
// at a time (the batched worker, whose register budget has no room for the
// four-wide form)
// s_hi0: Shi holds the high words of the neighbour sums from staging index
// s_hi0 on (the sums below have none); with own counts in 64 bits, an output
// whose T'' block lies below s_hi0 takes 64 x 64-bit products. tx_lds: the
// level's term descriptors copied to LDS (level_term_words), else read from L.
template <int ILP>
__device__ inline void combine_outputs(const CombineArgs &A, int64_t v, int cv, const uint64_t *Xlo,
                                       const uint64_t *Slo, const uint64_t *Xhi, const uint64_t *Shi, bool owide,
                                       bool wide, int s_hi0, const uint16_t *tx_lds)
{
    const DevLut &L = *A.L;
    const int lane = threadIdx.x;
    const int h = A.h;
    const int Wh = L.W[h];
    // one descriptor and one key per output (see DevLut::out): few table reads per lane
    const uint32_t ob = L.out_off[h];
    const uint16_t *okey = L.out_key[cv] + ob;
    uint32_t cnt = 0;
    u128 nsum = 0;
    uint16_t *sk = A.slot_key + (size_t)v * A.W;
    uint64_t *sl = A.slot_lo + (size_t)v * A.W;
    uint64_t *sh = owide ? A.slot_hi + (size_t)v * A.W : nullptr;
    for (int o0 = 0; o0 < Wh; o0 += WAVE) {
        const int o = o0 + lane;
        u128 val = 0;
        const uint64_t d = o < Wh ? L.out[ob + o] : 0ull;
        if (o < Wh && !(A.bal && !(d >> 63))) {
            const int xb = (int)(d & 0xffffu), sb = (int)((d >> 16) & 0xffffu), tb = (int)((d >> 32) & 0xffffu);
            const int nsplit = (int)((d >> 48) & 0xffu);
            u128 acc = 0;
            // terms four at a time: the four descriptors, then all their LDS
            // operands, are requested before any product, so that the loads of
            // a group overlap instead of one latency per term
            const uint16_t *txs = tx_lds ? tx_lds + (tb - L.term_base[h][1]) : L.term_xs + tb;
            const int n4 = ILP >= 4 ? (nsplit & ~3) : 0;
            if (!owide) {
                uint64_t a64 = 0;
                for (int i = 0; i < n4; i += 4) {
                    uint32_t xs[4];
                    uint64_t xv[4], sv[4];
#pragma unroll
                    for (int j = 0; j < 4; j++) xs[j] = txs[i + j];
#pragma unroll
                    for (int j = 0; j < 4; j++) { xv[j] = Xlo[xb + (xs[j] & 0xffu)]; sv[j] = Slo[sb + (xs[j] >> 8)]; }
#pragma unroll
                    for (int j = 0; j < 4; j++) a64 += xv[j] * sv[j];
                }
                for (int i = n4; i < nsplit; i++) {
                    const uint32_t xs = txs[i];
                    a64 += Xlo[xb + (xs & 0xffu)] * Slo[sb + (xs >> 8)];
                }
                acc = a64;
            } else if (!wide || (!Xhi && sb < s_hi0)) {
                for (int i = 0; i < n4; i += 4) {
                    uint32_t xs[4];
                    uint64_t xv[4], sv[4];
#pragma unroll
                    for (int j = 0; j < 4; j++) xs[j] = txs[i + j];
#pragma unroll
                    for (int j = 0; j < 4; j++) { xv[j] = Xlo[xb + (xs[j] & 0xffu)]; sv[j] = Slo[sb + (xs[j] >> 8)]; }
#pragma unroll
                    for (int j = 0; j < 4; j++) acc += (u128)xv[j] * sv[j];
                }
                for (int i = n4; i < nsplit; i++) {
                    const uint32_t xs = txs[i];
                    acc += (u128)Xlo[xb + (xs & 0xffu)] * Slo[sb + (xs >> 8)];
                }
            } else if (!Xhi) {
                // own counts in 64 bits, neighbour sums in 128
                for (int i = 0; i < n4; i += 4) {
                    uint32_t xs[4];
                    uint64_t xv[4], sl[4], sh2[4];
#pragma unroll
                    for (int j = 0; j < 4; j++) xs[j] = txs[i + j];
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const int si = sb + (int)(xs[j] >> 8);
                        xv[j] = Xlo[xb + (xs[j] & 0xffu)];
                        sl[j] = Slo[si];
                        sh2[j] = Shi[si - s_hi0];
                    }
#pragma unroll
                    for (int j = 0; j < 4; j++) acc += mul_64x128(xv[j], mk128(sl[j], sh2[j]));
                }
                for (int i = n4; i < nsplit; i++) {
                    const uint32_t xs = txs[i];
                    const int xi = xb + (int)(xs & 0xffu), si = sb + (int)(xs >> 8);
                    acc += mul_64x128(Xlo[xi], mk128(Slo[si], Shi[si - s_hi0]));
                }
            } else {
                for (int i = 0; i < nsplit; i++) {
                    const uint32_t xs = txs[i];
                    const int xi = xb + (int)(xs & 0xffu), si = sb + (int)(xs >> 8);
                    u128 x = mk128(Xlo[xi], Xhi[xi]), s = mk128(Slo[si], Shi[si]);
                    acc += x * s;
                }
            }
            const uint32_t beta = (uint32_t)((d >> 56) & 0x7fu);
            // beta divides the sum exactly (Eq. (1) counts each copy beta times): the
            // level kernels divide by a modular inverse; the batched worker keeps
            // the long division, which needs fewer registers there
            if (beta == 1) val = acc;
            else if (ILP >= 4) val = owide ? div_exact_small(acc, beta) : (u128)div_exact_small64(lo64(acc), beta);
            else val = div_small(acc, beta);
        }
        const bool nz = val != 0;
        const uint64_t bal = __ballot(nz);
        // output o is dense position o of the vertex's colour, so this round's
        // ballot is word o0 / 64 of its presence bitmap
        if (A.bm && lane == 0) A.bm[(size_t)v * A.BW + (o0 >> 6)] = bal;
        if (nz) {
            const uint32_t pos = cnt + (uint32_t)__popcll(bal & lanemask_lt());
            sk[pos] = okey[o];
            sl[pos] = lo64(val);
            if (owide) sh[pos] = hi64(val);
            nsum += val;
        }
        cnt += (uint32_t)__popcll(bal);
    }
    nsum = wave_sum128(nsum);
    if (lane == 0) {
        A.meta[v] = cnt | (owide ? 0x80000000u : 0u);
        A.Nout[v] = nsum;
    }
}

// Copies nwords 64-bit words from global memory to LDS with direct-to-LDS dword
// loads (lane l moves dword l of each block of 64): the data never occupies
// registers. The loads count in vmcnt like any other; wait before reading dst.
__device__ inline void lds_dma_words(const uint64_t *src, uint64_t *dst, int nwords)
{
    const int lane = threadIdx.x;
    const int nd = 2 * nwords;
    for (int b = 0; b < nd; b += WAVE)
        if (b + lane < nd)
            __builtin_amdgcn_global_load_lds(
                (const __attribute__((address_space(1))) void *)((const uint32_t *)src + b + lane),
                (__attribute__((address_space(3))) void *)((uint32_t *)dst + b), 4, 0, 0);
}
// s_waitcnt vmcnt(0): every vector memory load of the wave, direct-to-LDS ones included, has landed
__device__ inline void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// The same counts with the loads ordered for latency: every load that depends
// on v alone goes out first (lane q <= PMAX takes level q's record handle and
// neighbour-sum bound; the neighbour sums themselves go to LDS, by direct
// loads with DMA, else through a register per lane and level), then the level
// sums and the first entry per lane of each own record, then the key index of
// those entries. A wave thus waits about two memory latencies before the
// products instead of one per dependent step. PMAX bounds the levels unrolled
// (PMAX >= h - 1); longer rows and records are finished by loops, and high
// words (wide) are staged by loops as well.
// DMA: the neighbour sums reach lo_area (LDS) by direct-to-LDS loads; HI_LDS:
// hi_area is LDS too, so their high words may go the same way (the batched
// worker's hi_area is global scratch: filled by ordinary stores)
template <bool SLOTS, int PMAX, bool DMA, bool HI_LDS = false>
__device__ inline void combine_vertex_pf(const CombineArgs &A, int64_t v, uint64_t *lo_area, uint64_t *hi_area,
                                         int *wide_list, int *wide_count, bool own_hi = true,
                                         const uint16_t *tx_lds = nullptr)
{
    const DevLut &L = *A.L;
    const int lane = threadIdx.x;
    const int h = A.h;
    int cv = 0;
    if (A.zero_only) {   // level k: colour-0 vertices only
        cv = A.g.colors[v];
        if (cv != 0) {
            if (lane == 0) { A.meta[v] = 0; A.Nout[v] = 0; }
            return;
        }
    }
    const int plo = A.bal ? 2 : 1, phi = A.bal ? h - 2 : h - 1;
    const int XT = L.xoff[h];
    uint64_t *Xlo = lo_area, *Slo = lo_area + XT;
    // own_hi false: hi_area holds the neighbour sums' high words only
    uint64_t *Xhi = own_hi ? hi_area : nullptr, *Shi = own_hi && hi_area ? hi_area + XT : hi_area;
    // the neighbour sums go to LDS at once, unless this is a listing pass (no
    // hi_area) at a level where many vertices will be listed for 128 bits
    // (late_dma): there the vertex first learns whether it stays (below), so
    // that a listed vertex loads nothing it will load again
    auto dma_sums = [&]() {
        for (int hs = 1; hs <= phi; hs++)
            if (A.Slo[hs]) lds_dma_words(A.Slo[hs] + (size_t)v * L.WS[hs], Slo + L.soff[hs], L.WS[hs]);
    };
    const bool late = DMA && !hi_area && A.late_dma;
    if (DMA && !late) dma_sums();
    if (!A.zero_only) cv = A.g.colors[v];
    // lane q: handle of v's level-q record (q >= 2) and M_q(v) (0: sums not built)
    // packed levels of one bitmap word also give each lane q that word: bit l marks
    // dense position l, and the entry there is the popcount of the bits below l
    const uint64_t *locp = nullptr, *poolp = nullptr, *bmp = nullptr;
    const uint32_t *metap = nullptr;
    const u128 *Np = nullptr, *mp = nullptr;
#pragma unroll
    for (int q = 1; q <= PMAX; q++)
        if (lane == q && q <= phi) {
            mp = A.M[q];
            if (q >= 2) {
                if (SLOTS) { metap = A.lev[q].meta; Np = A.lev[q].N; }
                else {
                    locp = A.lev[q].P.loc; poolp = A.lev[q].P.pool;
                    if (A.lev[q].P.BW == 1) bmp = A.lev[q].P.bm;
                }
            }
        }
    uint64_t hd = 0;
    if (SLOTS) hd = ((uint64_t)v << 32) | (metap ? metap[v] : 0u);
    else hd = locp ? locp[v] : 0ull;
    const uint64_t bmw = bmp ? bmp[v] : 0ull;
    const u128 Mq = mp ? mp[v] : (u128)0;
    uint64_t sw[PMAX + 1];
#pragma unroll
    for (int q = 1; q <= PMAX; q++) {
        sw[q] = 0;
        if (!DMA && q <= phi && A.Slo[q] && lane < L.WS[q]) sw[q] = A.Slo[q][(size_t)v * L.WS[q] + lane];
    }
    u128 Nq = 0;
    if (h_len<SLOTS>(hd)) {
        if (SLOTS) Nq = Np[v];
        else { const uint64_t *rp = poolp + LOC_OFF(hd); Nq = mk128(rp[0], rp[1]); }
    }
    uint32_t ek[PMAX + 1];
    uint64_t el[PMAX + 1];
#pragma unroll
    for (int q = 2; q <= PMAX; q++) {
        ek[q] = 0;
        el[q] = 0;
        if (q <= phi) {
            const RecView<SLOTS> r = h_rec<SLOTS>(A.lev[q], readlane64(hd, q));
            if (!SLOTS && A.lev[q].P.BW == 1) {
                const uint64_t word = readlane64(bmw, q);
                if ((word >> lane) & 1ull) el[q] = r.lo[__popcll(word & ((1ull << lane) - 1ull))];
            } else if ((uint32_t)lane < r.len) {
                ek[q] = r.key[lane];
                el[q] = r.lo[lane];
            }
        }
    }
    // bound: lane hp contributes N_hp(v) M_{h-hp}(v) (level 1: N = 1)
    const u128 Mpair = shfl128(Mq, (h - lane) & (WAVE - 1));
    u128 term = 0;
    if (lane >= plo && lane <= phi) term = sat_mul(lane == 1 ? (u128)1 : Nq, Mpair);
    const u128 U = wave_satsum128(term);
    if (U == ~(u128)0 || bitlen128(U) > A.max_bits) {
        if (DMA) wait_vm_all();   // no load may land in LDS after the area is handed on
        if (lane == 0) { atomicOr(A.err, 1); A.meta[v] = 0; A.Nout[v] = 0; }
        return;
    }
    const bool owide = hi64(U) != 0;
    bool wide = false, xwide = false;
    uint64_t smask = 0;   // bit q: the level-q neighbour sums have high words
    if (owide) {
        xwide = __ballot(lane >= 2 && lane <= phi && h_wide<SLOTS>(hd)) != 0;
        smask = __ballot(lane >= 1 && lane <= phi && hi64(Mq) != 0);
        wide = xwide || smask != 0;
    }
    if (wide && !hi_area) {
        // own records with high words: from the back of the list (wide_count[2]);
        // neighbour sums alone: from the front (wide_count[0])
        if (DMA) wait_vm_all();
        if (lane == 0) {
            if (xwide) wide_list[A.g.n - 1 - atomicAdd(wide_count + 2, 1)] = (int)v;
            else wide_list[atomicAdd(wide_count, 1)] = (int)v;
        }
        return;
    }
    // own counts in 64 bits: high words are staged from the lowest sum level that
    // has them (hs_hi), at the start of hi_area
    const int hs_hi = Xhi || !smask ? 1 : __builtin_ctzll(smask);
    const int s_hi0 = L.soff[hs_hi];
    if (wide && A.hi_cap > 0 && L.soff[phi + 1] - s_hi0 > A.hi_cap) {
        // a launch sized for fewer high words than this vertex has (not expected:
        // the listing applies the same test)
        if (DMA) wait_vm_all();
        if (lane == 0) { atomicOr(A.err, 4); A.meta[v] = 0; A.Nout[v] = 0; }
        return;
    }
    if (late) dma_sums();
    const bool stage_xhi = wide && Xhi;
    for (int i = lane; i < XT; i += WAVE) {
        Xlo[i] = 0;
        if (stage_xhi) Xhi[i] = 0;
    }
    if (!DMA) {
#pragma unroll
        for (int q = 1; q <= PMAX; q++)
            if (q <= phi && A.Slo[q] && lane < L.WS[q]) Slo[L.soff[q] + lane] = sw[q];
    }
    for (int hs = 1; hs <= phi; hs++) {
        if (!A.Slo[hs]) continue;
        const int ws = L.WS[hs];
        const uint64_t *gl = A.Slo[hs] + (size_t)v * ws;
        if (!DMA)
            for (int i = WAVE + lane; i < ws; i += WAVE) Slo[L.soff[hs] + i] = gl[i];
        if (wide && hs >= hs_hi) {
            const bool sw128 = hi64(A.M[hs][v]) != 0;
            const uint64_t *gh = sw128 ? A.Shi[hs] + hi_row(A.Shrow[hs], v) * ws : nullptr;
            uint64_t *dst = Shi + (L.soff[hs] - s_hi0);
            if (DMA && HI_LDS && sw128) lds_dma_words(gh, dst, ws);
            else
                for (int i = lane; i < ws; i += WAVE) dst[i] = sw128 ? gh[i] : 0;
        }
    }
    __syncthreads();
    if (lane == 0) Xlo[L.xoff[1]] = 1;   // level 1: the single node, coloured c_v
    const int16_t *xidx = A.key_xidx + (size_t)cv * L.nkeys;
#pragma unroll
    for (int q = 2; q <= PMAX; q++) {
        if (q > phi) continue;
        const RecView<SLOTS> r = h_rec<SLOTS>(A.lev[q], readlane64(hd, q));
        if (!SLOTS && A.lev[q].P.BW == 1) {
            if ((readlane64(bmw, q) >> lane) & 1ull) Xlo[L.xoff[q] + lane] = el[q];
        } else if ((uint32_t)lane < r.len) {
            Xlo[L.xoff[q] + xidx[ek[q]]] = el[q];
        }
        if (stage_xhi) {
            for (uint32_t e = lane; e < r.len; e += WAVE) {
                const int x = L.xoff[q] + xidx[r.key[e]];
                if (e >= WAVE) Xlo[x] = r.lo[e];
                Xhi[x] = r.hi ? r.hi[e] : 0;
            }
        } else if (r.len > WAVE) {
            // the entries past the first 64, four per lane with their loads issued
            // before any store
            for (uint32_t e0 = WAVE + lane; e0 < r.len; e0 += 4 * WAVE) {
                uint32_t kx[4];
                uint64_t lx[4];
                int xi[4];
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const uint32_t e = e0 + j * WAVE;
                    kx[j] = e < r.len ? r.key[e] : 0u;
                    lx[j] = e < r.len ? r.lo[e] : 0ull;
                }
#pragma unroll
                for (int j = 0; j < 4; j++) xi[j] = e0 + j * WAVE < r.len ? xidx[kx[j]] : 0;
#pragma unroll
                for (int j = 0; j < 4; j++)
                    if (e0 + j * WAVE < r.len) Xlo[L.xoff[q] + xi[j]] = lx[j];
            }
        }
    }
    if (DMA) wait_vm_all();
    __syncthreads();
    combine_outputs<SLOTS ? 1 : 4>(A, v, cv, Xlo, Slo, stage_xhi ? Xhi : nullptr, Shi, owide, wide, s_hi0, tx_lds);
}

// one workgroup per vertex, low words in LDS; vertices that need 128 bits are
// listed for k_combine_wide
// eight waves per SIMD (one register below the compiler's own choice): the
// combine waits on memory, and the extra waves measured 9 % faster
template <int PMAX>
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(8, 8))) k_combine(CombineArgs A, int *wide_list, int *wide_count)
{
    extern __shared__ uint64_t sm[];
    if ((int64_t)blockIdx.x < A.g.n) combine_vertex_pf<false, PMAX, true>(A, blockIdx.x, sm, nullptr, wide_list, wide_count);
}

// the listed vertices only (level k under zero-rooting: the colour-0 vertices)
template <int PMAX>
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(8, 8))) k_combine_list(CombineArgs A, const int32_t *rows, int *wide_list, int *wide_count)
{
    extern __shared__ uint64_t sm[];
    combine_vertex_pf<false, PMAX, true>(A, __builtin_amdgcn_readfirstlane(rows[blockIdx.x]), sm, nullptr, wide_list, wide_count);
}

// The combine of a level with at most 64 outputs per vertex, four vertices per
// wave (16 lanes each): such a vertex has few terms (k = 6: 40 and 45 outputs
// of 2 and 3 terms on average at levels 4 and 5), so one vertex per wave spends
// its time waiting on the loads that stage it; four groups overlap them. The
// rows (a list, else 0..nrows-1) whose bound U reaches 2^64 are listed in
// fallback (count[5]) for k_combine_list; the others end here as in
// combine_vertex_pf: slot, meta, N and the level's single bitmap word.
constexpr int CGL = 16;   // lanes per vertex of the grouped combine
__device__ inline uint64_t grp_shfl64(uint64_t x, int src) { return shfl64(x, (lane_id() & ~(CGL - 1)) + src); }
template <int PMAX>
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(8, 8))) k_combine_group(CombineArgs A, const int32_t *rows, int64_t nrows, int32_t *fallback, int *count)
{
    extern __shared__ uint64_t sm[];
    const DevLut &L = *A.L;
    const int lane = threadIdx.x, g = lane / CGL, s = lane % CGL;
    const int h = A.h;
    const int plo = A.bal ? 2 : 1, phi = A.bal ? h - 2 : h - 1;
    const int XT = L.xoff[h], ST = L.soff[h], Wh = L.W[h];
    uint64_t *Xlo = sm + (size_t)g * (XT + ST), *Slo = Xlo + XT;
    const int64_t i = (int64_t)blockIdx.x * (WAVE / CGL) + g;
    const bool in = i < nrows;
    const int64_t v = in ? (rows ? (int64_t)rows[i] : i) : 0;
    const int cv = in ? (int)A.g.colors[v] : 0;
    const bool act = in && !(A.zero_only && cv != 0);
    if (in && !act && s == 0) { A.meta[v] = 0; A.Nout[v] = 0; }
    // sub-lane q: the handle of v's level-q record (q >= 2) and M_q(v)
    const u128 *mp = nullptr;
    const uint64_t *locp = nullptr, *poolp = nullptr;
#pragma unroll
    for (int q = 1; q <= PMAX; q++)
        if (s == q && q <= phi) {
            mp = A.M[q];
            if (q >= 2) { locp = A.lev[q].P.loc; poolp = A.lev[q].P.pool; }
        }
    const uint64_t hd = act && locp ? locp[v] : 0ull;
    const u128 Mq = act && mp ? mp[v] : (u128)0;
    u128 Nq = 0;
    if (LOC_LEN(hd)) { const uint64_t *rp = poolp + LOC_OFF(hd); Nq = mk128(rp[0], rp[1]); }
    // bound: sub-lane hp contributes N_hp(v) M_{h-hp}(v) (level 1: N = 1), summed
    // (saturating) over the group
    const int pr = (h - s) & (CGL - 1);
    const u128 Mpair = mk128(grp_shfl64(lo64(Mq), pr), grp_shfl64(hi64(Mq), pr));
    u128 U = act && s >= plo && s <= phi ? sat_mul(s == 1 ? (u128)1 : Nq, Mpair) : (u128)0;
#pragma unroll
    for (int off = CGL / 2; off >= 1; off >>= 1)
        U = sat_add(U, mk128(shfl64(lo64(U), lane ^ off), shfl64(hi64(U), lane ^ off)));
    const bool ovf = U == ~(u128)0 || bitlen128(U) > A.max_bits;
    if (act && ovf && s == 0) { atomicOr(A.err, 1); A.meta[v] = 0; A.Nout[v] = 0; }
    const bool owide = hi64(U) != 0;
    const bool run = act && !ovf && !owide;
    const bool isfb = act && !ovf && owide && s == 0;
    const uint64_t fb = __ballot(isfb);
    int fbase = 0;
    if (lane == 0 && fb) fbase = atomicAdd(count + 5, __popcll(fb));
    fbase = __shfl(fbase, 0);
    if (isfb) fallback[fbase + __popcll(fb & lanemask_lt())] = (int32_t)v;
    // staging: own counts X (zeroed, then the records) and neighbour sums S
    if (run) {
        for (int j = s; j < XT; j += CGL) Xlo[j] = 0;
        for (int hs = 1; hs <= phi; hs++) {
            if (!A.Slo[hs]) continue;
            const int ws = L.WS[hs];
            const uint64_t *gl = A.Slo[hs] + (size_t)v * ws;
            for (int j = s; j < ws; j += CGL) Slo[L.soff[hs] + j] = gl[j];
        }
    }
    __syncthreads();
    const int16_t *xidx = A.key_xidx + (size_t)cv * L.nkeys;
    if (run && s == 0) Xlo[L.xoff[1]] = 1;
#pragma unroll
    for (int q = 2; q <= PMAX; q++) {
        const uint64_t hq = grp_shfl64(hd, q);
        if (!run || q > phi) continue;
        const RecView<false> r = h_rec<false>(A.lev[q], hq);
        // four entries per lane with their loads issued before any store
        for (uint32_t e0 = s; e0 < r.len; e0 += 4 * CGL) {
            uint32_t kx[4];
            uint64_t lx[4];
            int xi[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint32_t e = e0 + j * CGL;
                kx[j] = e < r.len ? r.key[e] : 0u;
                lx[j] = e < r.len ? r.lo[e] : 0ull;
            }
#pragma unroll
            for (int j = 0; j < 4; j++) xi[j] = e0 + j * CGL < r.len ? xidx[kx[j]] : 0;
#pragma unroll
            for (int j = 0; j < 4; j++)
                if (e0 + j * CGL < r.len) Xlo[L.xoff[q] + xi[j]] = lx[j];
        }
    }
    __syncthreads();
    // outputs o = s, s + 16, ... of the group's vertex, compacted in order
    const uint32_t ob = L.out_off[h];
    const uint16_t *okey = L.out_key[cv] + ob;
    uint16_t *sk = A.slot_key + (size_t)v * A.W;
    uint64_t *sl = A.slot_lo + (size_t)v * A.W;
    uint32_t cnt = 0;
    uint64_t nsum = 0, bmw = 0;
    for (int o0 = 0; o0 < Wh; o0 += CGL) {
        const int o = o0 + s;
        uint64_t val = 0;
        const uint64_t d = run && o < Wh ? L.out[ob + o] : 0ull;
        if (run && o < Wh && !(A.bal && !(d >> 63))) {
            const int xb = (int)(d & 0xffffu), sb = (int)((d >> 16) & 0xffffu), tb = (int)((d >> 32) & 0xffffu);
            const int nsplit = (int)((d >> 48) & 0xffu);
            const uint16_t *txs = L.term_xs + tb;
            uint64_t a64 = 0;
            for (int t = 0; t < nsplit; t++) {
                const uint32_t xs = txs[t];
                a64 += Xlo[xb + (xs & 0xffu)] * Slo[sb + (xs >> 8)];
            }
            const uint32_t beta = (uint32_t)((d >> 56) & 0x7fu);
            val = beta == 1 ? a64 : div_exact_small64(a64, beta);
        }
        const bool nz = val != 0;
        const uint32_t gm = (uint32_t)(__ballot(nz) >> (g * CGL)) & 0xffffu;
        if (nz) {
            const uint32_t pos = cnt + (uint32_t)__popc(gm & ((1u << s) - 1u));
            sk[pos] = okey[o];
            sl[pos] = val;
            nsum += val;
        }
        bmw |= (uint64_t)gm << o0;
        cnt += (uint32_t)__popc(gm);
    }
#pragma unroll
    for (int off = CGL / 2; off >= 1; off >>= 1) nsum += shfl64(nsum, lane ^ off);
    if (run && s == 0) {
        A.meta[v] = cnt;
        A.Nout[v] = nsum;
        if (A.bm) A.bm[(size_t)v * A.BW] = bmw;
    }
}

// The combine's width test alone, one vertex per lane (rows: a row list, else
// vertices 0..nrows-1). At levels where most vertices need 128-bit inputs, a
// wave per vertex that only learns this would hold a combine's LDS while it
// waits on the same few loads. Same bound U and tests as combine_vertex_pf: an
// overflowing vertex is flagged, one with U = 0 has no nonzero output and is
// finished here, and the rest are listed: 64-bit inputs at the front of
// narrow (count[5]); high words in the top-level neighbour sums only at its
// back (count[6]); in lower-level sums too at the front of wide_list
// (count[0]); own records with high words at its back (count[2]).
__global__ void __launch_bounds__(256) k_combine_classify(CombineArgs A, const int32_t *rows, int64_t nrows,
                                                          int32_t *narrow, int *wide_list, int *count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i < nrows;
    const int64_t v = in ? (rows ? (int64_t)rows[i] : i) : 0;
    const int h = A.h;
    const int plo = A.bal ? 2 : 1, phi = A.bal ? h - 2 : h - 1;
    int cls = -1;   // 0 narrow, 1 front of wide_list, 2 its back, 3 back of narrow
    if (in) {
        u128 N[SCC_KMAX], M[SCC_KMAX];
        bool xwide = false, mwide = false, lower = false;
#pragma unroll
        for (int q = 1; q < SCC_KMAX; q++) {
            N[q] = 1;
            M[q] = 0;
            if (q > phi) continue;
            if (q >= 2) {
                const uint64_t hd = A.lev[q].P.loc[v];
                xwide |= h_wide<false>(hd);
                N[q] = h_N<false>(A.lev[q], hd);
            }
            if (A.M[q]) M[q] = A.M[q][v];
            mwide |= hi64(M[q]) != 0;
            lower |= q < phi && hi64(M[q]) != 0;
        }
        u128 U = 0;
#pragma unroll
        for (int hp = 1; hp < SCC_KMAX; hp++) {
            if (hp < plo || hp > phi) continue;
            u128 Mp = 0;   // M[h - hp], picked without a dynamic register index
#pragma unroll
            for (int q = 1; q < SCC_KMAX; q++)
                if (q + hp == h) Mp = M[q];
            U = sat_add(U, sat_mul(N[hp], Mp));
        }
        if (U == ~(u128)0 || bitlen128(U) > A.max_bits) {
            atomicOr(A.err, 1);
            A.meta[v] = 0;
            A.Nout[v] = 0;
        } else if (U == 0) {
            A.meta[v] = 0;
            A.Nout[v] = 0;
        } else {
            const bool wide = hi64(U) != 0 && (xwide || mwide);
            cls = !wide ? 0 : (xwide ? 2 : (lower ? 1 : 3));
        }
    }
    // one atomic per wave and list
    const uint64_t b0 = __ballot(cls == 0), b1 = __ballot(cls == 1), b2 = __ballot(cls == 2), b3 = __ballot(cls == 3);
    int base0 = 0, base1 = 0, base2 = 0, base3 = 0;
    if (lane_id() == 0) {
        if (b0) base0 = atomicAdd(count + 5, __popcll(b0));
        if (b1) base1 = atomicAdd(count, __popcll(b1));
        if (b2) base2 = atomicAdd(count + 2, __popcll(b2));
        if (b3) base3 = atomicAdd(count + 6, __popcll(b3));
    }
    base0 = __shfl(base0, 0);
    base1 = __shfl(base1, 0);
    base2 = __shfl(base2, 0);
    base3 = __shfl(base3, 0);
    const uint64_t below = lanemask_lt();
    if (cls == 0) narrow[base0 + __popcll(b0 & below)] = (int32_t)v;
    else if (cls == 1) wide_list[base1 + __popcll(b1 & below)] = (int)v;
    else if (cls == 2) wide_list[A.g.n - 1 - (base2 + __popcll(b2 & below))] = (int)v;
    else if (cls == 3) narrow[A.g.n - 1 - (base3 + __popcll(b3 & below))] = (int32_t)v;
}

// the listed vertices, with high words in LDS as well. OWN: vertices whose own
// records have high words, listed from the back of wide_list (lds = 2 (xoff_h +
// soff_h) words); else vertices with high words in neighbour sums only, listed
// from the front, which stage just those (lds = xoff_h + 2 soff_h words) and so
// fit more waves per CU; BACK: such vertices listed from the back of the list
// (those with high words in the top-level sums only: lds = xoff_h + soff_h +
// WS_{h-1} words, A.hi_cap = WS_{h-1})
// The level's term descriptors of Eq. (1) (term_xs from term_base[h][1] on:
// binom(k-1, h-1) (2^(h-1) - 1) of them) as 64-bit words of LDS, rounded up to 8
__host__ __device__ inline int level_term_words(int k, int h)
{
    int b = 1;   // binom(k-1, h-1)
    for (int i = 0; i < h - 1; i++) b = b * (k - 1 - i) / (i + 1);
    const int n = b * ((1 << (h - 1)) - 1);
    return (n * 2 + 63) / 64 * 8;
}

// persistent over the listed vertices: the LDS holds the level's term
// descriptors (copied once), then each vertex's staging areas
template <bool OWN, bool BACK = OWN>
__global__ void __launch_bounds__(WAVE) k_combine_wide(CombineArgs A, const int *wide_list, const int *wide_count)
{
    extern __shared__ uint64_t sm[];
    const int cnt = __builtin_amdgcn_readfirstlane(*wide_count);
    if ((int)blockIdx.x >= cnt) return;
    const DevLut &L = *A.L;
    const int tw = level_term_words(L.k, A.h);
    uint16_t *tx = (uint16_t *)sm;
    const uint16_t *src = L.term_xs + L.term_base[A.h][1];
    for (int i = threadIdx.x; i < tw * 4; i += WAVE) tx[i] = src[i];
    uint64_t *lo = sm + tw;
    const int lo_words = L.xoff[A.h] + L.soff[A.h];
    __syncthreads();
    for (int i = blockIdx.x; i < cnt; i += gridDim.x) {
        const int v = __builtin_amdgcn_readfirstlane(BACK ? wide_list[A.g.n - 1 - i] : wide_list[i]);
        combine_vertex_pf<false, SCC_KMAX - 1, true, true>(A, v, lo, lo + lo_words, nullptr, nullptr, OWN, tx);
        __syncthreads();
    }
}

// stored entries and 128-bit vertices of a level
__global__ void __launch_bounds__(256) k_meta_sum(int64_t n, const uint32_t *meta, unsigned long long *out)
{
    __shared__ uint64_t part[2][256 / WAVE];
    uint64_t len = 0, wide = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t m = meta[v];
        len += META_LEN(m);
        wide += META_WIDE(m);
    }
    len = wave_sum64(len);
    wide = wave_sum64(wide);
    if (lane_id() == 0) { part[0][threadIdx.x / WAVE] = len; part[1][threadIdx.x / WAVE] = wide; }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0, b = 0;
        for (int w = 0; w < 256 / WAVE; w++) { a += part[0][w]; b += part[1][w]; }
        if (a) atomicAdd(&out[0], (unsigned long long)a);
        if (b) atomicAdd(&out[1], (unsigned long long)b);
    }
}

// record size in 64-bit words
__global__ void k_words(int64_t n, const uint32_t *meta, uint64_t *words)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    uint32_t m = meta[v], len = META_LEN(m);
    words[v] = len ? (uint64_t)REC_HDR + key_words(len) + (uint64_t)len * (META_WIDE(m) ? 2u : 1u) : 0;
}

// Packing: each vertex's slot is copied into the pool at its offset, in one
// pass that can also set the presence bitmap (bit = position in the dense level-h
// layout) from the keys. Records are short, so 16 lanes take one vertex and a
// wave packs four at a time. Returns the vertex's (stored entries, 128-bit flag) in lane 0 of its
// group.
struct PackView {
    int64_t n;
    int W, BW, nkeys;
    const uint32_t *meta;
    const uint64_t *off_incl;        // inclusive running sums of record sizes
    const uint16_t *skey;
    const uint64_t *slo, *shi;
    const u128 *N;
    uint64_t *pool, *loc, *bm;
    const int16_t *key_xidx;
    const uint8_t *colors;
};

__device__ inline uint64_t rec_words(uint32_t m)
{
    const uint32_t len = META_LEN(m);
    return len ? (uint64_t)REC_HDR + key_words(len) + (uint64_t)len * (META_WIDE(m) ? 2u : 1u) : 0;
}

constexpr int PACK_ILP = 4;   // copies in flight per lane in pack_four
// BITS: also the presence bitmaps, from the keys (the level kernels' combine
// writes them itself)
template <bool BITS>
__device__ inline void pack_four(const PackView &P, int64_t v0, unsigned long long (*bits)[8], uint64_t &nlen,
                                 uint64_t &nwide)
{
    const int lane = threadIdx.x, g = lane >> 4, l = lane & 15;
    const int64_t v = v0 + g;
    const bool act = v < P.n;
    const uint32_t m = act ? P.meta[v] : 0u, len = META_LEN(m);
    if (act && l == 0) { nlen += len; nwide += META_WIDE(m); }
    if (BITS) {
        if (l < P.BW) bits[g][l] = 0;
        __syncthreads();
    }
    if (act) {
        const uint32_t kw = key_words(len);
        const uint64_t start = P.off_incl[v] - rec_words(m);
        if (l == 0) P.loc[v] = make_loc(start, len, META_WIDE(m));
        if (len) {
            uint64_t *rec = P.pool + start;
            if (l == 0) { rec[0] = lo64(P.N[v]); rec[1] = hi64(P.N[v]); }
            rec += REC_HDR;
            uint16_t *keys = (uint16_t *)rec;
            const int16_t *xi = P.key_xidx + (size_t)P.colors[v] * P.nkeys;
            const size_t base = (size_t)v * P.W;
            if (!BITS && (base & 3) == 0) {
                // four keys a word; past the record's end the word keeps zeros (the
                // slot words read there lie inside the slot array and its margin)
                const uint64_t *src = (const uint64_t *)(P.skey + base);
                for (uint32_t q0 = l; q0 < kw; q0 += 16 * PACK_ILP) {
                    uint64_t x[PACK_ILP];
#pragma unroll
                    for (int j = 0; j < PACK_ILP; j++) {
                        const uint32_t q = q0 + 16 * j;
                        x[j] = q < kw ? src[q] : 0ull;
                    }
#pragma unroll
                    for (int j = 0; j < PACK_ILP; j++) {
                        const uint32_t q = q0 + 16 * j;
                        if (q >= kw) continue;
                        const uint32_t rem = len - 4 * q;   // >= 1
                        rec[q] = rem < 4 ? x[j] & ((1ull << (16 * rem)) - 1ull) : x[j];
                    }
                }
            } else {
                for (uint32_t e = l; e < kw * 4; e += 16) {
                    uint16_t key = 0;
                    if (e < len) {
                        key = P.skey[base + e];
                        if (BITS) {
                            const int li = xi[key];
                            if (li >= 0) atomicOr(&bits[g][li >> 6], 1ull << (li & 63));
                        }
                    }
                    keys[e] = key;
                }
            }
            // PACK_ILP loads of a lane in flight before its stores (the compiler
            // cannot move a load above a store to the pool by itself)
            for (int part = 0; part < (META_WIDE(m) ? 2 : 1); part++) {
                const uint64_t *src = (part ? P.shi : P.slo) + base;
                uint64_t *dst = rec + kw + (part ? len : 0u);
                for (uint32_t e0 = l; e0 < len; e0 += 16 * PACK_ILP) {
                    uint64_t x[PACK_ILP];
#pragma unroll
                    for (int j = 0; j < PACK_ILP; j++) {
                        const uint32_t e = e0 + 16 * j;
                        x[j] = e < len ? src[e] : 0ull;
                    }
#pragma unroll
                    for (int j = 0; j < PACK_ILP; j++) {
                        const uint32_t e = e0 + 16 * j;
                        if (e < len) dst[e] = x[j];
                    }
                }
            }
        }
    }
    if (BITS) {
        __syncthreads();
        if (act && l < P.BW) P.bm[(size_t)v * P.BW + l] = bits[g][l];
        __syncthreads();
    }
}

// BITS: the level's combine did not set the bitmaps (the dedicated level-2 and
// level-3 kernels)
template <bool BITS>
__global__ void __launch_bounds__(WAVE) k_pack(PackView P)
{
    __shared__ unsigned long long bits[4][8];   // BW <= ceil(420 / 64)
    uint64_t nlen = 0, nwide = 0;
    for (int64_t v0 = (int64_t)blockIdx.x * 4; v0 < P.n; v0 += (int64_t)gridDim.x * 4)
        pack_four<BITS>(P, v0, bits, nlen, nwide);
}

// ---------------------------------------------------------------------------
// Level-k totals: eta_v (all shapes) and per-block partial sums per unrooted shape
// ---------------------------------------------------------------------------
constexpr int TOT_WAVES = 4;   // waves per block of k_totals
// one wave per vertex, strided over the grid: the lanes take the record's
// entries (one pass), eta_v is their wave sum, and each entry's count goes to
// its unrooted shape's 128-bit sum in the wave's LDS (64-bit atomics, the
// carry into the high word)
__global__ void __launch_bounds__(TOT_WAVES * WAVE) k_totals(GraphView g, const DevLut *Lp, LevelView Lk, int zero_only,
                                                             u128 *eta, u128 *part)
{
    __shared__ unsigned long long acc[TOT_WAVES][32][2];
    const DevLut &L = *Lp;
    const int w = threadIdx.x / WAVE, lane = lane_id();
    const int nu = L.num_unr;
    if (lane < 32) acc[w][lane][0] = acc[w][lane][1] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * TOT_WAVES;
    for (int64_t v = (int64_t)blockIdx.x * TOT_WAVES + w; v < g.n; v += stride) {
        Rec r{nullptr, 0, 0, false, false};
        if (!zero_only || g.colors[v] == 0) r = rec_of(Lk, v);
        u128 e = 0;
        for (uint32_t q = lane; q < r.len; q += WAVE) {
            const int t = (int)(r.key(q) - L.off[L.k]) / L.bk[L.k];
            const int j = L.unr_of[t];
            const u128 c = r.cnt(q);
            e += c;
            const unsigned long long lo = lo64(c), old = atomicAdd(&acc[w][j][0], lo);
            const unsigned long long hi = hi64(c) + (old + lo < old ? 1ull : 0ull);
            if (hi) atomicAdd(&acc[w][j][1], hi);
        }
        e = wave_sum128(e);
        if (lane == 0) eta[v] = e;
    }
    __syncthreads();
    if ((int)threadIdx.x < nu) {
        u128 s = 0;
        for (int q = 0; q < TOT_WAVES; q++) s += mk128(acc[q][threadIdx.x][0], acc[q][threadIdx.x][1]);
        part[(size_t)blockIdx.x * 32 + threadIdx.x] = s;
    }
}

__global__ void __launch_bounds__(256) k_reduce_parts(const u128 *part, int nb, int nu, u128 *out)
{
    __shared__ u128 ws[256 / WAVE];
    const int j = blockIdx.x;
    if (j >= nu) return;
    u128 s = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[(size_t)b * 32 + j];
    s = wave_sum128(s);
    if (lane_id() == 0) ws[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        u128 t = 0;
        for (int w = 0; w < 256 / WAVE; w++) t += ws[w];
        out[j] = t;
    }
}

// ---------------------------------------------------------------------------
// Variable-length counts (Sec. 3.3): re-encoding of a finished level. Pass 1
// sizes every record in the new layout, a scan places them, pass 2 writes
// them: per chunk of 64 entries a wave scan of the byte lengths gives each
// count's offset.
// ---------------------------------------------------------------------------
__device__ inline uint32_t vlc_rec_words(uint32_t len, uint64_t bytes)
{
    return len ? (uint32_t)(REC_HDR + key_words(len) + vlc_ck_words(len) + (bytes + 7) / 8) : 0u;
}

__global__ void __launch_bounds__(WAVE) k_vlc_size(int64_t n, LevelView L, uint64_t *words)
{
    for (int64_t v = blockIdx.x; v < n; v += gridDim.x) {
        const Rec r = rec_of(L, v);
        uint64_t b = 0;
        for (uint32_t e = threadIdx.x; e < r.len; e += WAVE) b += vlc_bytes(r.cnt(e));
        b = wave_sum64(b);
        if (threadIdx.x == 0) words[v] = vlc_rec_words(r.len, b);
    }
}

__global__ void __launch_bounds__(WAVE) k_vlc_write(int64_t n, LevelView L, const uint64_t *incl, uint64_t *pool,
                                                    uint64_t *loc)
{
    const int lane = threadIdx.x;
    for (int64_t v = blockIdx.x; v < n; v += gridDim.x) {
        const Rec r = rec_of(L, v);
        const uint64_t start = v ? incl[v - 1] : 0;
        if (lane == 0) loc[v] = make_loc(start, r.len, 0);
        if (!r.len) continue;
        uint64_t *p = pool + start;
        if (lane < 2) p[lane] = r.p[lane];   // level sum N
        uint16_t *hd = (uint16_t *)(p + REC_HDR);
        uint16_t *ck = (uint16_t *)(p + REC_HDR + key_words(r.len));
        uint8_t *cb = (uint8_t *)(p + REC_HDR + key_words(r.len) + vlc_ck_words(r.len));
        uint32_t base = 0;
        for (uint32_t e0 = 0; e0 < r.len; e0 += WAVE) {
            const uint32_t e = e0 + lane;
            u128 c = 0;
            uint32_t l = 0;
            if (e < r.len) {
                c = r.cnt(e);
                l = vlc_bytes(c);
            }
            const uint32_t incl_l = wave_incl_scan32(l);
            const uint32_t off = base + incl_l - l;
            if (e < r.len) {
                hd[e] = (uint16_t)(r.key(e) | (l << 11));
                if (e % VLC_CK == 0) ck[e / VLC_CK] = (uint16_t)off;
                for (uint32_t i = 0; i < l; i++) cb[off + i] = (uint8_t)(c >> (8 * i));
            }
            base += __shfl(incl_l, WAVE - 1, WAVE);
        }
    }
}

// Round skipping (Sec. 3.3): the uncoloured k-stars centred at v, binom(d_v, k-1),
// by the exact recurrence c_i = c_{i-1} (d - r + i) / i; flags a product that
// does not fit 128 bits
__global__ void k_star_weight(GraphView g, int r, u128 *w, unsigned long long *flag)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    const int64_t d = g.row_ptr[v + 1] - g.row_ptr[v];
    u128 c = d >= r ? 1 : 0;
    for (int i = 1; i <= r && c; i++) {
        const u128 p = sat_mul(c, (u128)(d - r + i));
        if (p == ~(u128)0) { atomicOr(flag, 1ull); c = 0; break; }
        c = div_small(p, (uint32_t)i);
    }
    w[v] = c;
}

// a running sum wrapped modulo 2^128 exactly where it decreases
__global__ void k_wrap_check(const u128 *pre, int64_t n, unsigned long long *flag)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= 1 && v < n && pre[v] < pre[v - 1]) atomicOr(flag, 1ull);
}

__global__ void k_eta_shape(GraphView g, const DevLut *Lp, LevelView Lk, int zero_only, int shape, u128 *eta)
{
    const DevLut &L = *Lp;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n) return;
    u128 e = 0;
    if (!zero_only || g.colors[v] == 0) {
        const Rec r = rec_of(Lk, v);
        for (uint32_t q = 0; q < r.len; q++) {
            const int t = (int)(r.key(q) - L.off[L.k]) / L.bk[L.k];
            if (L.unr_of[t] == shape) e += r.cnt(q);
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

// ---------------------------------------------------------------------------
// Packing many (instance, level) jobs at once (the batched build): record sizes
// and their running sums, then the records, with one launch per step for all
// jobs (blockIdx.y = job).
// ---------------------------------------------------------------------------
struct PackJobDev {
    int64_t n;
    int W, BW, nkeys, pad;
    const uint32_t *meta;
    uint64_t *words;                 // out: inclusive running sums of record sizes
    uint64_t *bsum;                  // scan scratch, one per SCAN_TILE vertices
    const uint16_t *skey;
    const uint64_t *slo, *shi;
    const u128 *N;
    uint64_t *pool, *loc, *bm;
    const int16_t *key_xidx;
    const uint8_t *colors;
    unsigned long long *stats;       // [0] stored entries, [1] 128-bit vertices (added to)
    uint64_t *total;                 // out: pool words
};

__global__ void __launch_bounds__(SCAN_T) k_mpack_sums(const PackJobDev *Js)
{
    __shared__ uint64_t sh[SCAN_T / WAVE];
    const PackJobDev J = Js[blockIdx.y];
    const int64_t nb = (J.n + SCAN_TILE - 1) / SCAN_TILE;
    if ((int64_t)blockIdx.x >= nb) return;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    uint64_t s = 0;
    for (int i = 0; i < SCAN_I; i++) {
        const int64_t idx = base + (int64_t)threadIdx.x * SCAN_I + i;
        if (idx < J.n) s += rec_words(J.meta[idx]);
    }
    const uint64_t incl = block_incl_scan<uint64_t>(s, sh);
    if (threadIdx.x == SCAN_T - 1) J.bsum[blockIdx.x] = incl;
}

__global__ void __launch_bounds__(SCAN_T) k_mpack_top(const PackJobDev *Js)
{
    __shared__ uint64_t sh[SCAN_T / WAVE];
    __shared__ uint64_t carry;
    const PackJobDev J = Js[blockIdx.x];
    const int64_t nb = (J.n + SCAN_TILE - 1) / SCAN_TILE;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += SCAN_T) {
        const int64_t idx = base + threadIdx.x;
        const uint64_t x = idx < nb ? J.bsum[idx] : 0;
        const uint64_t incl = block_incl_scan<uint64_t>(x, sh);
        const uint64_t c = carry;
        if (idx < nb) J.bsum[idx] = c + incl - x;
        __syncthreads();
        if (threadIdx.x == SCAN_T - 1) carry = c + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) *J.total = carry;
}

__global__ void __launch_bounds__(SCAN_T) k_mpack_apply(const PackJobDev *Js)
{
    __shared__ uint64_t sh[SCAN_T / WAVE];
    const PackJobDev J = Js[blockIdx.y];
    const int64_t nb = (J.n + SCAN_TILE - 1) / SCAN_TILE;
    if ((int64_t)blockIdx.x >= nb) return;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_I;
    uint64_t v[SCAN_I];
    uint64_t s = 0;
    for (int i = 0; i < SCAN_I; i++) {
        v[i] = (base + i < J.n) ? rec_words(J.meta[base + i]) : 0;
        s += v[i];
    }
    const uint64_t incl = block_incl_scan<uint64_t>(s, sh);
    uint64_t run = J.bsum[blockIdx.x] + incl - s;
    for (int i = 0; i < SCAN_I; i++) {
        run += v[i];
        if (base + i < J.n) J.words[base + i] = run;
    }
}

// the records of every job (as k_pack), plus the level's stored entries and
// 128-bit vertices
__global__ void __launch_bounds__(WAVE) k_mpack(const PackJobDev *Js)
{
    __shared__ unsigned long long bits[4][8];
    const PackJobDev J = Js[blockIdx.y];
    PackView P{J.n, J.W, J.BW, J.nkeys, J.meta, J.words, J.skey, J.slo, J.shi, J.N, J.pool, J.loc, J.bm,
               J.key_xidx, J.colors};
    uint64_t nlen = 0, nwide = 0;
    for (int64_t v0 = (int64_t)blockIdx.x * 4; v0 < J.n; v0 += (int64_t)gridDim.x * 4)
        pack_four<true>(P, v0, bits, nlen, nwide);
    nlen = wave_sum64(nlen);
    nwide = wave_sum64(nwide);
    if (threadIdx.x == 0 && nlen) atomicAdd(&J.stats[0], (unsigned long long)nlen);
    if (threadIdx.x == 0 && nwide) atomicAdd(&J.stats[1], (unsigned long long)nwide);
}

template <typename T>
scc_status scan_incl(scc_table *T_, const T *in, T *out, int64_t n)
{
    if (n <= 0) return SCC_OK;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    DevMem m = T_->mem;        // scratch ordered on the stream the scan runs on
    m.stream = T_->stream;
    T *bsum = (T *)m.get(nb * sizeof(T));
    if (!bsum) return set_error(SCC_ENOMEM, "scan scratch");
    hipLaunchKernelGGL(k_scan_sums<T>, dim3((unsigned)nb), dim3(SCAN_T), 0, T_->stream, in, n, bsum);
    hipLaunchKernelGGL(k_scan_top<T>, dim3(1), dim3(SCAN_T), 0, T_->stream, bsum, nb);
    hipLaunchKernelGGL(k_scan_apply<T>, dim3((unsigned)nb), dim3(SCAN_T), 0, T_->stream, in, out, n, bsum);
    m.put(bsum);   // stream-ordered release: reused only by later work on this stream
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(SCC_EDEVICE, "scan: %s", hipGetErrorString(e));
    return SCC_OK;
}

// grid-stride grids of one-wave workgroups, for kernels with even per-vertex work
// (uneven ones, gather and combine, launch one workgroup per vertex and let the
// dispatcher balance them)
unsigned grid_of(int64_t n) { return (unsigned)std::min<int64_t>(n, 256 * 80); }

LevelView view(const TableLevel &l)
{
    return LevelView{l.pool, l.loc, l.bm, l.BW, l.vlc ? 1 : 0};
}

LevelSrc packed_src(const TableLevel &l)
{
    LevelSrc s{};
    s.P = view(l);
    return s;
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
// one workgroup per vertex, or per listed vertex (rows non-null)
// Level 2 of Eq. (1) has one term per output: an edge rooted at v with colour set
// {c_v, j} has c = S_1(v)[j] copies (beta = 1), below 2^31. One thread per vertex
// writes the nonzero ones into v's slot in output order (ascending key), as the
// general combine would.
__global__ void __launch_bounds__(256) k_combine_level2(CombineArgs A)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= A.g.n) return;
    const DevLut &L = *A.L;
    const int cv = A.g.colors[v];
    const int W = L.W[2];
    const uint64_t *s1 = A.Slo[1] + (size_t)v * W;          // S_1 has W_2 = k - 1 entries
    const uint16_t *okey = L.out_key[cv] + L.out_off[2];
    uint16_t *sk = A.slot_key + (size_t)v * A.W;
    uint64_t *sl = A.slot_lo + (size_t)v * A.W;
    uint32_t cnt = 0;
    uint64_t sum = 0;
    for (int o = 0; o < W; o++) {
        const uint64_t c = s1[o];
        if (!c) continue;
        sk[cnt] = okey[o];
        sl[cnt] = c;
        cnt++;
        sum += c;
    }
    A.meta[v] = cnt;
    A.Nout[v] = sum;
}

// Level 3 of Eq. (1) reads only dense arrays: its own counts are X_1 = 1 and
// X_2, which equals S_1 entry for entry (an edge rooted at v with colours
// {c_v, j} has S_1(v)[j] copies), and its neighbour sums are S_1 and S_2. One
// thread per vertex evaluates the outputs from the same descriptors and terms
// as the general combine, in output order. The bound N_1 M_2 + N_2 M_1 is at
// most 2m + d_v^2, so 128 bits always suffice; a vertex whose S_2 needs high
// words is listed for the 128-bit combine instead.
__global__ void __launch_bounds__(256) k_combine_level3(CombineArgs A, int *wide_list, int *wide_count)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= A.g.n) return;
    const DevLut &L = *A.L;
    const int cv = A.g.colors[v];
    const int k1 = L.WS[1];                                  // k - 1
    if (hi64(A.M[2][v]) != 0) {
        wide_list[atomicAdd(wide_count, 1)] = (int)v;
        return;
    }
    const uint64_t *s1 = A.Slo[1] + (size_t)v * k1;
    const uint64_t *s2 = A.Slo[2] + (size_t)v * L.WS[2];
    uint64_t n2 = 0;
    for (int j = 0; j < k1; j++) n2 += s1[j];
    const u128 U = (u128)lo64(A.M[2][v]) + (u128)n2 * lo64(A.M[1][v]);
    const bool owide = hi64(U) != 0;
    if (bitlen128(U) > A.max_bits) {
        atomicOr(A.err, 1);
        A.meta[v] = 0;
        A.Nout[v] = 0;
        return;
    }
    const uint32_t ob = L.out_off[3];
    const uint16_t *okey = L.out_key[cv] + ob;
    uint16_t *sk = A.slot_key + (size_t)v * A.W;
    uint64_t *sl = A.slot_lo + (size_t)v * A.W;
    uint64_t *sh = A.slot_hi + (size_t)v * A.W;
    uint32_t cnt = 0;
    u128 nsum = 0;
    for (int o = 0; o < L.W[3]; o++) {
        const uint64_t d = L.out[ob + o];
        const int xb = (int)(d & 0xffffu), sb = (int)((d >> 16) & 0xffffu), tb = (int)((d >> 32) & 0xffffu);
        const int nsplit = (int)((d >> 48) & 0xffu);
        const uint32_t beta = (uint32_t)((d >> 56) & 0x7fu);
        u128 acc = 0;
        for (int i = 0; i < nsplit; i++) {
            const uint32_t xs = L.term_xs[tb + i];
            const int xi = xb + (int)(xs & 0xffu), si = sb + (int)(xs >> 8);
            const uint64_t x = xi == 0 ? 1ull : s1[xi - 1];      // staging: [X_1 | X_2]
            const uint64_t sv = si < k1 ? s1[si] : s2[si - k1];  // staging: [S_1 | S_2]
            acc += (u128)x * sv;
        }
        const u128 val = beta == 1 ? acc : div_exact_small(acc, beta);
        if (val == 0) continue;
        sk[cnt] = okey[o];
        sl[cnt] = lo64(val);
        if (owide) sh[cnt] = hi64(val);
        cnt++;
        nsum += val;
    }
    A.meta[v] = cnt | (owide ? 0x80000000u : 0u);
    A.Nout[v] = nsum;
}

template <int PMAX>
static void launch_combine(const CombineArgs &C, int64_t n, const int32_t *rows, int64_t nrows, size_t lds,
                           hipStream_t st, int *wide_list, int *wide_count)
{
    if (rows) {
        if (nrows)
            hipLaunchKernelGGL(k_combine_list<PMAX>, dim3((unsigned)nrows), dim3(WAVE), lds, st, C, rows, wide_list,
                               wide_count);
    } else {
        hipLaunchKernelGGL(k_combine<PMAX>, dim3((unsigned)n), dim3(WAVE), lds, st, C, wide_list, wide_count);
    }
}

static scc_status build_levels(scc_table *T)
{
    const DevLut &HL = T->hlut;
    const int k = T->k;
    const int64_t n = T->n;
    hipStream_t st = T->stream;
    GraphView g{n, T->row_ptr, T->col_idx, T->colors};
    const bool zero = T->rooting == SCC_ROOT_ZERO;
    // round skipping (Sec. 3.3): level k-1 is not built, and of the neighbour sums
    // above level k-3 only those the designated decompositions use (|T''| = hs)
    const bool bal = T->rooting == SCC_ROOT_BALANCED;
    bool s_need[SCC_KMAX + 1];
    for (int hs = 0; hs <= SCC_KMAX; hs++) s_need[hs] = !bal || hs <= k - 3;
    for (int q = 0; bal && q < HL.r[k]; q++)
        if (HL.designated[q]) s_need[k - HL.dec_hp[k][q]] = true;
    const int hub_degree = T->hub_degree;

    // [0] flags, [1] 128-bit vertices with high words in neighbour sums only,
    // [2] wide gather rows, [3] 128-bit vertices whose own records have high
    // words; bytes 16..23 receive a level's pool size, so that one read returns
    // it with the flags. A high-word array released while its copy is still
    // queued is safe: the allocator hooks free in the table's stream order
    // (hipFree, without hooks, waits for the device).
    // [0] flags; [1], [3] combine lists; [2] gather's wide rows; [4..5] pool size;
    // [6], [7] combine lists; [8..9] heavy degree (u64); [10] gather's narrow rows
    int *err = (int *)T->mem.get(64);
    std::vector<void *> scratch{err};
    struct Guard {
        scc_table *T; std::vector<void *> *s;
        ~Guard() { for (void *p : *s) T->mem.put(p); }
    } guard{T, &scratch};
    auto get = [&](size_t bytes) { void *p = T->mem.get(bytes); if (p) scratch.push_back(p); return p; };
    if (!err) return set_error(SCC_ENOMEM, "flags");
    int32_t *gwide = (int32_t *)get((size_t)n * 4 + 256);   // rows whose neighbour sums need 128 bits
    if (!gwide) return set_error(SCC_ENOMEM, "wide rows");

    // per-level start/end events (whole level, and its gather), read once at the end
    // and the start of its combine (which ends with the level)
    hipEvent_t ev[SCC_KMAX + 1][2] = {}, gev[SCC_KMAX + 1][2] = {}, cev[SCC_KMAX + 1] = {};
    struct EvGuard {
        hipEvent_t (*a)[2], (*b)[2], *c;
        ~EvGuard() {
            for (int h = 0; h <= SCC_KMAX; h++) {
                for (int j = 0; j < 2; j++) {
                    if (a[h][j]) (void)hipEventDestroy(a[h][j]);
                    if (b[h][j]) (void)hipEventDestroy(b[h][j]);
                }
                if (c[h]) (void)hipEventDestroy(c[h]);
            }
        }
    } evg{ev, gev, cev};
    for (int h = 1; h <= k; h++) {
        for (int j = 0; j < 2; j++) {
            HIP_TRY(hipEventCreate(&ev[h][j]));
            HIP_TRY(hipEventCreate(&gev[h][j]));
        }
        HIP_TRY(hipEventCreate(&cev[h]));
    }

    // hub rows and their neighbour chunks, and the rows between the grouped
    // low-degree ones and the hubs (the same for every level)
    int nhub = 0, nmid = 0, nzero = 0;
    int64_t low_rows = 0;
    int32_t *hubs = nullptr, *mids = nullptr, *zrows = nullptr;
    int32_t *chunk_v = nullptr, *chunk_q = nullptr;
    int64_t *chunk_e = nullptr;
    int64_t nchunk = 0;
    bool fused = false;   // hub running sums built with the gather
    if (n) {
        hubs = (int32_t *)get((size_t)n * 4 + 8);
        mids = (int32_t *)get((size_t)n * 4 + 8);
        zrows = (int32_t *)get((size_t)n * 4 + 8);
        if (!hubs || !mids || !zrows) return set_error(SCC_ENOMEM, "row lists");
        HIP_TRY(hipMemsetAsync(err, 0, 16, st));
        hipLaunchKernelGGL(k_row_lists, dim3((unsigned)((n + ROW_LIST_T - 1) / ROW_LIST_T)), dim3(ROW_LIST_T), 0, st, g,
                           hub_degree, hubs, mids, zrows, err);
        int cnt[4] = {0, 0, 0, 0};
        HIP_TRY(hipMemcpyAsync(cnt, err, 16, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        nhub = cnt[0];
        nmid = cnt[1];
        low_rows = cnt[2];
        nzero = cnt[3];
    }
    if (nhub) {
        std::vector<int32_t> hh(nhub);
        std::vector<int64_t> rp(2 * (size_t)nhub);
        HIP_TRY(hipMemcpyAsync(hh.data(), hubs, (size_t)nhub * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        std::sort(hh.begin(), hh.end());
        int64_t *rows = (int64_t *)get((size_t)nhub * 16 + 16);
        if (!rows) return set_error(SCC_ENOMEM, "hub rows");
        HIP_TRY(hipMemcpyAsync(hubs, hh.data(), (size_t)nhub * 4, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_hub_rows, dim3((unsigned)((nhub + 255) / 256)), dim3(256), 0, st, g, hubs, nhub, rows);
        HIP_TRY(hipMemcpyAsync(rp.data(), rows, (size_t)nhub * 16, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        // the sampler's hub running sums come with the gather when every hub's
        // blocks fit the budget: chunks are then single blocks of HUB_BLOCK
        std::vector<int64_t> poff((size_t)nhub * (SCC_KMAX + 1), 0);
        int64_t at = 0;
        for (int i = 0; i < nhub; i++) {
            const int64_t nb = (rp[2 * i + 1] - rp[2 * i] + HUB_BLOCK - 1) / HUB_BLOCK;
            for (int h = 1; h < k; h++) {
                poff[(size_t)i * (SCC_KMAX + 1) + h] = at;
                if (h == 1 || s_need[h]) at += 2 * (int64_t)HL.WS[h] * nb;
            }
        }
        fused = at * 8 <= T->hub_prefix_budget;
        if (fused) {
            T->hub_chunk = (int)HUB_BLOCK;
            T->hub_pre = (uint64_t *)T->alloc((size_t)at * 8 + 8);
            T->hub_poff = (int64_t *)T->alloc(poff.size() * 8);
            T->hub_index = (int32_t *)T->alloc((size_t)n * 4 + 4);
            if (!T->hub_pre || !T->hub_poff || !T->hub_index)
                return set_error(SCC_ENOMEM, "hub running sums (%lld bytes)", (long long)at * 8);
            HIP_TRY(hipMemcpyAsync(T->hub_poff, poff.data(), poff.size() * 8, hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemsetAsync(T->hub_index, 0xff, (size_t)n * 4 + 4, st));
            hipLaunchKernelGGL(k_set_rows, dim3((unsigned)((nhub + 255) / 256)), dim3(256), 0, st, T->hub_index, hubs,
                               (const int *)nullptr, (int64_t)nhub, 0);
        }
        std::vector<int32_t> cv, cq;
        std::vector<int64_t> ce;
        for (int i = 0; i < nhub; i++)
            for (int64_t e = rp[2 * i]; e < rp[2 * i + 1]; e += T->hub_chunk) {
                cv.push_back(hh[i]);
                ce.push_back(e);
                cq.push_back(i);
            }
        nchunk = (int64_t)cv.size();
        chunk_v = (int32_t *)get(cv.size() * 4 + 8);
        chunk_e = (int64_t *)get(ce.size() * 8 + 8);
        chunk_q = (int32_t *)get(cq.size() * 4 + 8);
        if (!chunk_v || !chunk_e || !chunk_q) return set_error(SCC_ENOMEM, "hub chunks");
        HIP_TRY(hipMemcpyAsync(chunk_v, cv.data(), cv.size() * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(chunk_e, ce.data(), ce.size() * 8, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(chunk_q, cq.data(), cq.size() * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
        T->hub_host.assign(hh.begin(), hh.end());
        T->hub_rows_host = rp;
    }
    T->nhub = nhub;

    // level 1 neighbour sums
    TableSums &S1 = T->S[1];
    S1.lo = (uint64_t *)T->alloc((size_t)n * (k - 1) * 8 + 8);
    S1.M = (u128 *)T->alloc((size_t)n * 16 + 16);
    if (!S1.lo || !S1.M) return set_error(SCC_ENOMEM, "level-1 sums");
    HIP_TRY(hipEventRecord(ev[1][0], st));
    if (n)
        hipLaunchKernelGGL(k_gather1, dim3(grid_of((n + WAVE - 1) / WAVE)), dim3(WAVE), 0, st, g, k, S1.lo, S1.M,
                           (int64_t)(nhub ? hub_degree : INT64_MAX));
    if (nhub)
        hipLaunchKernelGGL(k_gather1_hub, dim3((unsigned)nchunk), dim3(WAVE), 0, st, g, k, chunk_v, chunk_e, T->hub_chunk,
                           S1.lo);
    if (fused) {
        hipLaunchKernelGGL(k_hub_l1_blocks, dim3((unsigned)nchunk), dim3(WAVE), 0, st, g, k, hubs, chunk_e, chunk_q,
                           T->hub_pre, T->hub_poff);
        hipLaunchKernelGGL(k_hub_block_scan, dim3((unsigned)((int64_t)nhub * (k - 1))), dim3(WAVE), 0, st, g, hubs,
                           k - 1, 1, 0, S1.M, T->hub_pre, T->hub_poff);
    }
    HIP_TRY(hipEventRecord(ev[1][1], st));
    T->gather_bytes[1] = (double)n * 8.0 + (double)T->nnz_g * 5.0 + (double)n * (k - 1) * 8.0;

    // scratch slots for the combine, sized for the widest level
    int maxW = 0;
    for (int h = 2; h <= k; h++) maxW = std::max(maxW, HL.W[h]);
    uint16_t *slot_key = (uint16_t *)get((size_t)n * maxW * 2 + 256);
    uint64_t *slot_lo = (uint64_t *)get((size_t)n * maxW * 8 + 256);
    uint64_t *slot_hi = (uint64_t *)get((size_t)n * maxW * 8 + 256);
    uint64_t *words = (uint64_t *)get((size_t)n * 8 + 256);
    uint32_t *meta = (uint32_t *)get((size_t)n * 4 + 256);
    u128 *Nsc = (u128 *)get((size_t)n * 16 + 256);
    int *wide_list = (int *)get((size_t)n * 4 + 256);
    // row lists of one level: the gather's 64-bit rows where its rows are sorted,
    // then the combine's 64-bit vertices (width test per lane) or the grouped
    // combine's vertices whose bound reaches 2^64
    int32_t *narrow = (int32_t *)get((size_t)n * 4 + 256);
    if (!slot_key || !slot_lo || !slot_hi || !words || !meta || !Nsc || !wide_list || !narrow)
        return set_error(SCC_ENOMEM, "combine scratch (%lld bytes)", (long long)n * maxW * 18);

    int64_t heavy_prev = 0;   // sum of degrees of the vertices whose previous-level N has a high word
    for (int h = 2; h <= k; h++) {
        const bool last = h == k;
        int64_t top_wide_rows = 0;   // rows of the sums gathered now whose high words exist
        HIP_TRY(hipEventRecord(ev[h][0], st));
        HIP_TRY(hipMemsetAsync(err, 0, 64, st));   // flags and the level's counts of listed rows
        const int hs = h - 1;   // neighbour sums needed now
        if (hs >= 2 && s_need[hs]) {
            TableSums &Sx = T->S[hs];
            const size_t sz = (size_t)n * HL.WS[hs] * 8;
            Sx.M = (u128 *)T->alloc((size_t)n * 16 + 16);
            Sx.lo = (uint64_t *)T->alloc(sz + 8);
            Sx.hrow = (int32_t *)T->alloc((size_t)n * 4 + 8);
            if (!Sx.M || !Sx.lo || !Sx.hrow) return set_error(SCC_ENOMEM, "neighbour sums level %d (%zu bytes)", hs, sz);
            HIP_TRY(hipMemsetAsync(Sx.hrow, 0xff, (size_t)n * 4 + 8, st));
            GatherArgs G{};
            G.g = g; G.k = k; G.nkeys = HL.nkeys; G.WS = HL.WS[hs]; G.rows_zero = zero && h == k;
            G.key_lo = HL.off[hs]; G.key_n = HL.r[hs] * HL.bk[hs];
            G.hub_degree = hub_degree;
            G.L = packed_src(T->lev[hs]); G.M = Sx.M; G.key_sidx = T->key_sidx; G.Slo = Sx.lo; G.Shi = nullptr;
            G.chunk_v = chunk_v; G.chunk_e = chunk_e; G.err = err;
            G.Lut = T->dlut; G.hs = hs; G.bk1 = HL.bk1[hs];
            G.hrow = Sx.hrow; G.wide_rows = gwide; G.wide_count = err + 2;
            if (fused) { G.hub_pre = T->hub_pre; G.hub_poff = T->hub_poff; G.chunk_q = chunk_q; }
            const size_t lds = gather_lds(HL.WS[hs]);
            const int gs = group_size(HL.WS[hs]);
            const int64_t ngroups = (n + gs - 1) / gs;
            HIP_TRY(hipEventRecord(gev[hs][0], st));
            // grouped low-degree rows pay off while records are short; long records
            // fill a wave from a few neighbours already
            const bool grouped = T->gather_mode == SCC_GATHER_GROUPED ||
                                 (T->gather_mode == SCC_GATHER_AUTO && n && 2 * low_rows >= n &&
                                  T->lev[hs].pool_words <= (uint64_t)GROUP_WORDS * n);
            if (grouped) {
                if (nmid) hipLaunchKernelGGL(k_gather_list, dim3((unsigned)nmid), dim3(WAVE), lds, st, G, mids);
                if (n)
                    hipLaunchKernelGGL(k_gather_group, dim3((unsigned)std::min<int64_t>(ngroups, 16384)), dim3(WAVE),
                                       group_lds(HL.WS[hs], gs), st, G, gs);
            } else if (G.rows_zero) {
                if (nzero) hipLaunchKernelGGL(k_gather_list, dim3((unsigned)nzero), dim3(WAVE), lds, st, G, zrows);
            } else if (n && heavy_prev * 8 > n) {
                // many rows border a vertex whose level sum needs 128 bits: sort the
                // rows out first (one per lane), then the 64-bit pass takes the others only
                T->sorted_sum_rows |= 1 << hs;
                hipLaunchKernelGGL(k_gather_classify, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, G, Nsc,
                                   narrow, err + 10);
                int nn = 0;
                HIP_TRY(hipMemcpyAsync(&nn, err + 10, 4, hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                if (nn) hipLaunchKernelGGL(k_gather_list, dim3((unsigned)nn), dim3(WAVE), lds, st, G, narrow);
            } else if (n) {
                hipLaunchKernelGGL(k_gather, dim3((unsigned)n), dim3(WAVE), lds, st, G);
            }
            // high words only for the hubs (merged across chunks) and the listed
            // rows whose bound reaches 2^64, in compact rows: hubs first. The hubs'
            // rows are known now, so their gather runs while the count of wide
            // rows comes back; with wide rows the array grows and the hub rows move.
            const size_t row_bytes = (size_t)HL.WS[hs] * 8;
            Sx.hi_rows = nhub;
            Sx.hi = (uint64_t *)T->alloc((size_t)nhub * row_bytes + 8);
            if (!Sx.hi) return set_error(SCC_ENOMEM, "neighbour sums level %d, high words", hs);
            G.Shi = Sx.hi;
            if (nhub) {
                hipLaunchKernelGGL(k_set_rows, dim3((unsigned)((nhub + 255) / 256)), dim3(256), 0, st, Sx.hrow, hubs,
                                   (const int *)nullptr, (int64_t)nhub, 0);
                hipLaunchKernelGGL(k_hub_prepare, dim3((unsigned)nhub), dim3(WAVE), 0, st, G, hubs);
                hipLaunchKernelGGL(k_gather_hub, dim3((unsigned)nchunk), dim3(WAVE), lds, st, G, T->hub_chunk);
            }
            int nw = 0;
            HIP_TRY(hipMemcpyAsync(&nw, err + 2, 4, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            top_wide_rows = (int64_t)nw + nhub;
            if (nw) {
                uint64_t *hi = (uint64_t *)T->alloc((size_t)(nhub + nw) * row_bytes + 8);
                if (!hi) return set_error(SCC_ENOMEM, "neighbour sums level %d, high words", hs);
                if (nhub) HIP_TRY(hipMemcpyAsync(hi, Sx.hi, (size_t)nhub * row_bytes, hipMemcpyDeviceToDevice, st));
                T->release(Sx.hi, (size_t)nhub * row_bytes + 8);
                Sx.hi = hi;
                Sx.hi_rows = (int64_t)nhub + nw;
                G.Shi = hi;
                hipLaunchKernelGGL(k_set_rows, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, Sx.hrow, gwide,
                                   (const int *)nullptr, (int64_t)nw, nhub);
                hipLaunchKernelGGL(k_gather_wide, dim3((unsigned)nw), dim3(WAVE), lds, st, G);
            }
            HIP_TRY(hipEventRecord(gev[hs][1], st));
            // the sampler's hub running sums of this level (not part of the gather)
            if (fused)
                hipLaunchKernelGGL(k_hub_block_scan, dim3((unsigned)((int64_t)nhub * HL.WS[hs])), dim3(WAVE), 0, st, g,
                                   hubs, HL.WS[hs], hs, G.rows_zero, Sx.M, T->hub_pre, T->hub_poff);
        }
        // combine into slots: a vertex needing 128 bits waits for the second kernel
        TableLevel &Lv = T->lev[h];
        Lv.loc = (uint64_t *)T->alloc((size_t)n * 8 + 8);
        if (!Lv.loc) return set_error(SCC_ENOMEM, "level %d locators", h);
        const bool skipped = bal && h == k - 1;
        if (!skipped) {
            // sized by the level's width alone: allocated while the GPU still works
            Lv.BW = (HL.W[h] + 63) / 64;
            Lv.bm = (uint64_t *)T->alloc((size_t)n * Lv.BW * 8 + 8);
            if (!Lv.bm) return set_error(SCC_ENOMEM, "level %d bitmaps", h);
            // the combine writes the words of the vertices it evaluates; the rest stay 0
            HIP_TRY(hipMemsetAsync(Lv.bm, 0, (size_t)n * Lv.BW * 8, st));
        }
        if (skipped) {
            // skipped level: every record empty (its entry count stays 0 in the summary)
            Lv.pool = (uint64_t *)T->alloc(64);
            if (!Lv.pool) return set_error(SCC_ENOMEM, "level %d", h);
            Lv.pool_words = 0;
            Lv.BW = 0;
            Lv.bm = nullptr;
            HIP_TRY(hipMemsetAsync(Lv.loc, 0, (size_t)n * 8 + 8, st));
            HIP_TRY(hipEventRecord(ev[h][1], st));
            continue;
        }
        HIP_TRY(hipEventRecord(cev[h], st));
        CombineArgs C{};
        C.g = g; C.L = T->dlut; C.h = h; C.zero_only = zero && last; C.max_bits = T->max_bits;
        C.bal = bal && last;
        for (int q = 2; q < h; q++) C.lev[q] = packed_src(T->lev[q]);
        for (int q = 1; q < h; q++) {
            C.Slo[q] = T->S[q].lo; C.Shi[q] = T->S[q].hi; C.Shrow[q] = T->S[q].hrow; C.M[q] = T->S[q].M;
        }
        C.key_xidx = T->key_xidx; C.W = HL.W[h];
        // many rows of the top sum level with high words: most vertices will be
        // listed for the 128-bit combine, so they are classified one per lane
        // first (a listing pass at levels 2 and 3 stages late instead)
        C.late_dma = 8 * top_wide_rows > n;
        C.slot_key = slot_key; C.slot_lo = slot_lo; C.slot_hi = slot_hi;
        C.meta = meta; C.Nout = Nsc; C.err = err;
        C.bm = Lv.bm; C.BW = Lv.BW;
        const size_t lds = (size_t)(HL.xoff[h] + HL.soff[h]) * 8;
        if (n) {
            // level k under zero-rooting: only the colour-0 vertices have records
            const bool zl = C.zero_only != 0;
            if (zl) {
                HIP_TRY(hipMemsetAsync(meta, 0, (size_t)n * 4, st));
                HIP_TRY(hipMemsetAsync(Nsc, 0, (size_t)n * 16, st));
            }
            const int phi = C.bal ? h - 2 : h - 1;
            const bool classified = h >= 4 && (T->width_test == SCC_WIDTH_PER_LANE ||
                                               (T->width_test == SCC_WIDTH_AUTO && C.late_dma));
            // at most 64 outputs per vertex: four vertices per wave
            const bool grouped = !classified && h >= 4 && HL.W[h] <= 64 && phi <= 5;
            if (classified) {
                T->lane_width_test |= 1 << h;
                // most vertices will need 128-bit inputs: the width test one vertex
                // per lane first, then the 64-bit combine of the narrow ones alone
                const int64_t nr = zl ? nzero : n;
                if (nr)
                    hipLaunchKernelGGL(k_combine_classify, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, C,
                                       zl ? zrows : nullptr, nr, narrow, wide_list, err + 1);
                int nn = 0;
                HIP_TRY(hipMemcpyAsync(&nn, err + 6, 4, hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                CombineArgs Cn = C;
                Cn.late_dma = 0;
                if (phi <= 3) launch_combine<3>(Cn, n, narrow, nn, lds, st, wide_list, err + 1);
                else if (phi <= 5) launch_combine<5>(Cn, n, narrow, nn, lds, st, wide_list, err + 1);
                else launch_combine<SCC_KMAX - 1>(Cn, n, narrow, nn, lds, st, wide_list, err + 1);
            } else if (grouped) {
                T->grouped_combine |= 1 << h;
                const int64_t nr = zl ? nzero : n;
                const size_t lds_g = (size_t)(WAVE / CGL) * (HL.xoff[h] + HL.soff[h]) * 8;
                if (nr) {
                    const dim3 grid((unsigned)((nr + WAVE / CGL - 1) / (WAVE / CGL)));
                    if (phi <= 3)
                        hipLaunchKernelGGL(k_combine_group<3>, grid, dim3(WAVE), lds_g, st, C, zl ? zrows : nullptr, nr,
                                           narrow, err + 1);
                    else
                        hipLaunchKernelGGL(k_combine_group<5>, grid, dim3(WAVE), lds_g, st, C, zl ? zrows : nullptr, nr,
                                           narrow, err + 1);
                }
                // the vertices whose bound reaches 2^64, one per wave
                int nf = 0;
                HIP_TRY(hipMemcpyAsync(&nf, err + 6, 4, hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                if (phi <= 3) launch_combine<3>(C, n, narrow, nf, lds, st, wide_list, err + 1);
                else launch_combine<5>(C, n, narrow, nf, lds, st, wide_list, err + 1);
            } else if (h == 2 && !zl && !C.bal)
                hipLaunchKernelGGL(k_combine_level2, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, C);
            else if (h == 3 && !zl && !C.bal)
                hipLaunchKernelGGL(k_combine_level3, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, C, wide_list,
                                   err + 1);
            else if (phi <= 3) launch_combine<3>(C, n, zl ? zrows : nullptr, nzero, lds, st, wide_list, err + 1);
            else if (phi <= 5) launch_combine<5>(C, n, zl ? zrows : nullptr, nzero, lds, st, wide_list, err + 1);
            else launch_combine<SCC_KMAX - 1>(C, n, zl ? zrows : nullptr, nzero, lds, st, wide_list, err + 1);
            // the 128-bit vertices (at k = 8 most of level 7, nearly all with high
            // words in neighbour sums only) stride over as many waves as each
            // kernel's LDS staging lets the chip hold
            int dev = 0, ncu = 0, per_s = 0, per_own = 0;
            const size_t ltw = (size_t)level_term_words(k, h) * 8;   // the level's term descriptors
            const size_t lds_s = (size_t)(HL.xoff[h] + 2 * HL.soff[h]) * 8 + ltw, lds_o = 2 * lds + ltw;
            HIP_TRY(hipGetDevice(&dev));
            HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
            HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_s, k_combine_wide<false>, WAVE, lds_s));
            HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_own, k_combine_wide<true>, WAVE, lds_o));
            const int64_t gs = std::min<int64_t>(n, std::max<int64_t>(1024, (int64_t)ncu * per_s));
            const int64_t go = std::min<int64_t>(n, std::max<int64_t>(1024, (int64_t)ncu * per_own));
            hipLaunchKernelGGL(k_combine_wide<false>, dim3((unsigned)gs), dim3(WAVE), lds_s, st, C, wide_list, err + 1);
            hipLaunchKernelGGL(k_combine_wide<true>, dim3((unsigned)go), dim3(WAVE), lds_o, st, C, wide_list, err + 3);
            if (classified) {
                // high words in the top-level sums only (listed at the back of narrow):
                // the high-word area holds that level alone, so more waves fit per CU
                CombineArgs Ct = C;
                Ct.hi_cap = HL.WS[phi];
                const size_t lds_t = (size_t)(HL.xoff[h] + HL.soff[h] + HL.WS[phi]) * 8 + ltw;
                int per_t = 0;
                HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_t, (k_combine_wide<false, true>), WAVE, lds_t));
                const int64_t gt = std::min<int64_t>(n, std::max<int64_t>(1024, (int64_t)ncu * per_t));
                hipLaunchKernelGGL((k_combine_wide<false, true>), dim3((unsigned)gt), dim3(WAVE), lds_t, st, Ct,
                                   (const int *)narrow, err + 7);
            }
        }
        if (n && !last)
            hipLaunchKernelGGL(k_heavy_degree, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 2048)), dim3(256), 0,
                               st, g, Nsc, (unsigned long long *)(err + 8));
        // record sizes and offsets; the pool size and the error flags in one read
        if (n) hipLaunchKernelGGL(k_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, meta, words);
        scc_status sst = scan_incl<uint64_t>(T, words, words, n);
        if (sst) return sst;
        struct { int f[4]; uint64_t total; int g[2]; uint64_t heavy; } hr{};   // the layout of err
        if (n) HIP_TRY(hipMemcpyAsync(err + 4, words + (n - 1), 8, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(&hr, err, sizeof hr, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const int *herr = hr.f;
        const uint64_t total = n ? hr.total : 0;
        if (herr[0] & 1) return set_error(SCC_EOVERFLOW, "a level-%d count needs more than %d bits", h, T->max_bits);
        if (herr[0] & 2) return set_error(SCC_EOVERFLOW, "a level-%d neighbour sum may exceed 128 bits", h);
        if (herr[0] & 4)
            return set_error(SCC_EDEVICE, "level %d: a vertex listed for the top-level 128-bit combine has more high words", h);
        heavy_prev = (int64_t)hr.heavy;
        T->wide_input_rows[h][0] = herr[1];
        T->wide_input_rows[h][1] = hr.g[1];
        T->wide_input_rows[h][2] = herr[3];
        Lv.pool_words = total;
        Lv.pool = (uint64_t *)T->alloc((size_t)total * 8 + 64);
        if (!Lv.pool) return set_error(SCC_ENOMEM, "level %d pool (%llu words)", h, (unsigned long long)total);
        if (n) {
            PackView P{n, HL.W[h], Lv.BW, HL.nkeys, meta, words, slot_key, slot_lo, slot_hi, Nsc, Lv.pool, Lv.loc,
                       Lv.bm, T->key_xidx, T->colors};
            // one group of four vertices per wave: the waves' dependent loads overlap.
            // The bitmaps come from the combine, except after the dedicated level-2
            // and level-3 kernels, which do not write them
            const bool bits = (h == 2 || h == 3) && !C.zero_only && !C.bal;
            if (bits) hipLaunchKernelGGL(k_pack<true>, dim3((unsigned)((n + 3) / 4)), dim3(WAVE), 0, st, P);
            else hipLaunchKernelGGL(k_pack<false>, dim3((unsigned)((n + 3) / 4)), dim3(WAVE), 0, st, P);
        }
        HIP_TRY(hipEventRecord(ev[h][1], st));
        if (n) hipLaunchKernelGGL(k_meta_sum, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0, st,
                                  n, meta, (unsigned long long *)T->dsum + 2 * h);
        HIP_TRY(hipGetLastError());
    }
    if (fused) {
        T->hub_count_pre = nhub;
        T->hubpre_ready = true;
    }
    // every level's duration (the stream is drained by the totals that follow)
    HIP_TRY(hipEventSynchronize(ev[k][1]));
    for (int h = 1; h <= k; h++) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, ev[h][0], ev[h][1]));
        T->level_ms[h] = ms;
        if (h == 1) T->gather_ms[1] = ms;
        if (h >= 2 && !(bal && h == k - 1)) {
            HIP_TRY(hipEventElapsedTime(&ms, cev[h], ev[h][1]));
            T->combine_ms[h] = ms;
        }
        if (h >= 2 && h < k && s_need[h]) {
            HIP_TRY(hipEventElapsedTime(&ms, gev[h][0], gev[h][1]));
            T->gather_ms[h] = ms;
        }
    }
    return SCC_OK;
}

// algorithmic bytes of each gather launch, computed after the build on request
static scc_status gather_stats(scc_table *T)
{
    if (T->stats_done) return SCC_OK;
    const int64_t n = T->n;
    hipStream_t st = T->stream;
    GraphView g{n, T->row_ptr, T->col_idx, T->colors};
    // one counter per level 0..k (the combine pass fills all of them)
    constexpr size_t ACC_BYTES = (SCC_KMAX + 1) * sizeof(unsigned long long);
    unsigned long long *acc = (unsigned long long *)T->mem.get(ACC_BYTES);
    if (!acc) return set_error(SCC_ENOMEM, "stats");
    for (int hs = 2; hs < T->k; hs++) {
        if (!T->S[hs].M) { T->gather_bytes[hs] = 0; continue; }   // not built (round skipping)
        HIP_TRY(hipMemsetAsync(acc, 0, 8, st));
        const bool rz = T->rooting == SCC_ROOT_ZERO && hs == T->k - 1;
        if (n) hipLaunchKernelGGL(k_gather_bytes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g,
                                  view(T->lev[hs]), T->S[hs].M, T->hlut.WS[hs], rz ? 1 : 0, acc);
        unsigned long long b = 0;
        HIP_TRY(hipMemcpyAsync(&b, acc, 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        T->gather_bytes[hs] = (double)b;
    }
    // the combine of every level and the level-k totals, in one counting pass
    HIP_TRY(hipMemsetAsync(acc, 0, ACC_BYTES, st));
    CombineBytesArgs A{};
    A.g = g; A.k = T->k; A.zero = T->rooting == SCC_ROOT_ZERO;
    for (int h = 2; h <= T->k; h++) A.lev[h] = view(T->lev[h]);
    for (int h = 1; h < T->k; h++) {
        A.WS[h] = h == 1 ? T->k - 1 : T->hlut.WS[h];
        A.s_built[h] = T->S[h].lo != nullptr;
        A.hrow[h] = T->S[h].hrow;
    }
    if (n) hipLaunchKernelGGL(k_combine_bytes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, acc);
    unsigned long long cb[SCC_KMAX + 1] = {0};
    static_assert(sizeof cb == ACC_BYTES, "one counter per level");
    HIP_TRY(hipMemcpyAsync(cb, acc, ACC_BYTES, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int h = 2; h <= T->k; h++) T->combine_bytes[h] = (double)cb[h];
    T->totals_bytes = (double)cb[0];
    T->mem.put(acc);
    T->stats_done = true;
    return SCC_OK;
}

// Level-k totals, launch half: eta and its running sums, the per-shape totals
// and the root total land in the device summary; nothing waits for the device.
constexpr int DSUM_TJ = 2 * (SCC_KMAX + 1);     // u64 index of the 32 per-shape totals
constexpr int DSUM_TOT = DSUM_TJ + 64;           // u64 index of the root total
constexpr int DSUM_STAR = DSUM_TOT + 2;          // uncoloured k-stars (round skipping)
constexpr int DSUM_SFLAG = DSUM_STAR + 2;        // nonzero: the star count overflowed
constexpr int DSUM_WORDS = DSUM_SFLAG + 1;

static scc_status totals_launch(scc_table *T)
{
    const int k = T->k;
    const int64_t n = T->n;
    hipStream_t st = T->stream;
    GraphView g{n, T->row_ptr, T->col_idx, T->colors};
    const bool zero = T->rooting == SCC_ROOT_ZERO;
    T->eta = (u128 *)T->alloc((size_t)n * 16 + 16);
    T->pre = (u128 *)T->alloc((size_t)n * 16 + 16);
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>((n + TOT_WAVES - 1) / TOT_WAVES, 8192));
    u128 *part = (u128 *)T->mem.get((size_t)nb * 32 * 16);
    if (!T->eta || !T->pre || !part) { T->mem.put(part); return set_error(SCC_ENOMEM, "totals"); }
    u128 *tjd = (u128 *)(T->dsum + DSUM_TJ);
    if (n)
        hipLaunchKernelGGL(k_totals, dim3((unsigned)nb), dim3(TOT_WAVES * WAVE), 0, st, g, T->dlut, view(T->lev[k]),
                           zero ? 1 : 0, T->eta, part);
    hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)T->hlut.num_unr), dim3(256), 0, st, part, (int)(n ? nb : 0),
                       T->hlut.num_unr, tjd);
    T->mem.put(part);   // stream-ordered
    scc_status s = scan_u128(T, T->eta, T->pre, n);
    if (s) return s;
    if (n) HIP_TRY(hipMemcpyAsync(T->dsum + DSUM_TOT, T->pre + (n - 1), 16, hipMemcpyDeviceToDevice, st));
    if (T->rooting == SCC_ROOT_BALANCED) {
        // stars: per-vertex counts, their running sums (the direct star sampler's
        // centre draw) and the total
        T->star_pre = (u128 *)T->alloc((size_t)n * 16 + 16);
        if (!T->star_pre) return set_error(SCC_ENOMEM, "star counts");
        unsigned long long *flag = (unsigned long long *)(T->dsum + DSUM_SFLAG);
        const unsigned blocks = (unsigned)((n + 255) / 256);
        if (n) hipLaunchKernelGGL(k_star_weight, dim3(blocks), dim3(256), 0, st, g, k - 1, T->star_pre, flag);
        s = scan_u128(T, T->star_pre, T->star_pre, n);
        if (s) return s;
        if (n) {
            hipLaunchKernelGGL(k_wrap_check, dim3(blocks), dim3(256), 0, st, T->star_pre, n, flag);
            HIP_TRY(hipMemcpyAsync(T->dsum + DSUM_STAR, T->star_pre + (n - 1), 16, hipMemcpyDeviceToDevice, st));
        }
    }
    HIP_TRY(hipGetLastError());
    return SCC_OK;
}

// finish half: one read of the device summary (waits for the table's stream)
static scc_status totals_finish(scc_table *T)
{
    uint64_t h[DSUM_WORDS];
    hipError_t e = hipMemcpyAsync(h, T->dsum, sizeof h, hipMemcpyDeviceToHost, T->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(T->stream);
    if (e != hipSuccess) return set_error(SCC_EDEVICE, "totals: %s", hipGetErrorString(e));
    const int k = T->k;
    const bool zero = T->rooting == SCC_ROOT_ZERO;
    for (int lv = 2; lv <= k; lv++) {
        T->lev[lv].nnz = (int64_t)h[2 * lv];
        T->lev[lv].wide = (int64_t)h[2 * lv + 1];
    }
    T->lev[1].nnz = T->n;
    const u128 tot = T->n ? mk128(h[DSUM_TOT], h[DSUM_TOT + 1]) : (u128)0;
    T->root_total = tot;
    if (T->rooting == SCC_ROOT_BALANCED) {
        // every copy of a non-star shape is counted once per node of its
        // designated rooting's orbit
        if (h[DSUM_SFLAG]) return set_error(SCC_EOVERFLOW, "the number of %d-stars needs more than 128 bits", k);
        T->stars = T->n ? mk128(h[DSUM_STAR], h[DSUM_STAR + 1]) : (u128)0;
        u128 t = 0;
        for (int j = 0; j < T->hlut.num_unr; j++) {
            const u128 tj = mk128(h[DSUM_TJ + 2 * j], h[DSUM_TJ + 2 * j + 1]);
            const int orb = T->hlut.bal_orbit[j];
            if (orb == 0) {
                if (tj) return set_error(SCC_EINVAL, "internal: counts of the star at level %d", k);
                T->tj[j] = 0;
                continue;
            }
            if (tj % (u128)orb) return set_error(SCC_EINVAL, "internal: shape %d total not divisible by its orbit", j);
            T->tj[j] = tj / (u128)orb;
            t += T->tj[j];
        }
        T->t = t;
        return SCC_OK;
    }
    for (int j = 0; j < T->hlut.num_unr; j++) {
        const u128 tj = mk128(h[DSUM_TJ + 2 * j], h[DSUM_TJ + 2 * j + 1]);
        T->tj[j] = zero ? tj : tj / (u128)k;
    }
    T->t = zero ? tot : tot / (u128)k;
    return SCC_OK;
}

static scc_status build_totals(scc_table *T)
{
    hipEvent_t e[2] = {};
    struct G { hipEvent_t *e; ~G() { for (int i = 0; i < 2; i++) if (e[i]) (void)hipEventDestroy(e[i]); } } gd{e};
    HIP_TRY(hipEventCreate(&e[0]));
    HIP_TRY(hipEventCreate(&e[1]));
    HIP_TRY(hipEventRecord(e[0], T->stream));
    scc_status s = totals_launch(T);
    if (s) return s;
    HIP_TRY(hipEventRecord(e[1], T->stream));
    s = totals_finish(T);
    if (s) return s;
    float ms = 0;
    HIP_TRY(hipEventSynchronize(e[1]));
    HIP_TRY(hipEventElapsedTime(&ms, e[0], e[1]));
    T->totals_ms = ms;
    return SCC_OK;
}

// Re-encodes every stored level with variable-length counts (Sec. 3.3). The
// sampler's running sums are prepared first, from the fixed layout; every
// reader after this point goes through the layout-aware record view.
static scc_status compact_levels(scc_table *T)
{
    scc_status s = prepare_all_sampling(T);
    if (s) return s;
    const int64_t n = T->n;
    hipStream_t st = T->stream;
    const unsigned grid = (unsigned)std::min<int64_t>(std::max<int64_t>(n, 1), 65536);
    for (int h = 2; h <= T->k; h++) {
        TableLevel &Lv = T->lev[h];
        uint64_t *words = (uint64_t *)T->mem.get((size_t)n * 8 + 8);
        if (!words) return set_error(SCC_ENOMEM, "record sizes");
        struct Put { scc_table *T; uint64_t *w; ~Put() { T->mem.put(w); } } put{T, words};
        if (n) hipLaunchKernelGGL(k_vlc_size, dim3(grid), dim3(WAVE), 0, st, n, view(Lv), words);
        s = scan_u64(T, words, words, n);
        if (s) return s;
        uint64_t total = 0;
        if (n) HIP_TRY(hipMemcpyAsync(&total, words + (n - 1), 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        uint64_t *pool = (uint64_t *)T->alloc((size_t)total * 8 + 64);
        uint64_t *loc = (uint64_t *)T->alloc((size_t)n * 8 + 8);
        if (!pool || !loc) return set_error(SCC_ENOMEM, "level %d variable-length records (%llu words)", h,
                                            (unsigned long long)total);
        if (n) hipLaunchKernelGGL(k_vlc_write, dim3(grid), dim3(WAVE), 0, st, n, view(Lv), words, pool, loc);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(st));
        T->release(Lv.pool, (size_t)Lv.pool_words * 8 + 64);
        T->release(Lv.loc, (size_t)n * 8 + 8);
        Lv.pool = pool;
        Lv.loc = loc;
        Lv.pool_words = total;
        Lv.vlc = true;
    }
    T->vlc = true;
    return SCC_OK;
}

static scc_status make_key_maps(scc_table *T)
{
    const DevLut &L = T->hlut;
    const int k = T->k;
    // both maps live in the table's host copy, so that their uploads need no wait here
    const size_t nk = (size_t)k * L.nkeys;
    T->key_maps_host.assign(2 * nk, (int16_t)-1);
    int16_t *sidx = T->key_maps_host.data(), *xidx = sidx + nk;
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
    T->key_sidx = (int16_t *)T->alloc(nk * 2);
    T->key_xidx = (int16_t *)T->alloc(nk * 2);
    T->dlut = (DevLut *)T->alloc(sizeof(DevLut));
    T->dsum = (uint64_t *)T->alloc(DSUM_WORDS * 8);
    if (!T->key_sidx || !T->key_xidx || !T->dlut || !T->dsum) return set_error(SCC_ENOMEM, "lookup tables");
    HIP_TRY(hipMemsetAsync(T->dsum, 0, DSUM_WORDS * 8, T->stream));
    HIP_TRY(hipMemcpyAsync(T->key_sidx, sidx, nk * 2, hipMemcpyHostToDevice, T->stream));
    HIP_TRY(hipMemcpyAsync(T->key_xidx, xidx, nk * 2, hipMemcpyHostToDevice, T->stream));
    HIP_TRY(hipMemcpyAsync(T->dlut, &T->hlut, sizeof(DevLut), hipMemcpyHostToDevice, T->stream));
    return SCC_OK;
}

static scc_table *new_table(const scc_csr *g, const uint8_t *colors, int k, const scc_build_opts &o);

// The table's graph on the device: a host graph (on_device = 0) and its
// colours are copied into memory the table owns; device pointers are borrowed.
static scc_status attach_graph(scc_table *T, const scc_csr *g, const uint8_t *colors)
{
    if (g->on_device) return SCC_OK;
    const int64_t n = g->n, nnz = g->nnz;
    int64_t *rp = (int64_t *)T->alloc((size_t)(n + 1) * 8);
    int32_t *ci = (int32_t *)T->alloc((size_t)std::max<int64_t>(nnz, 1) * 4);
    uint8_t *cl = (uint8_t *)T->alloc((size_t)std::max<int64_t>(n, 1));
    if (!rp || !ci || !cl) return set_error(SCC_ENOMEM, "graph copy");
    HIP_TRY(hipMemcpyAsync(rp, g->row_ptr, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, T->stream));
    if (nnz > 0) HIP_TRY(hipMemcpyAsync(ci, g->col_idx, (size_t)nnz * 4, hipMemcpyHostToDevice, T->stream));
    if (n > 0) HIP_TRY(hipMemcpyAsync(cl, colors, (size_t)n, hipMemcpyHostToDevice, T->stream));
    // the caller may free or change its host arrays once the call returns
    HIP_TRY(hipStreamSynchronize(T->stream));
    T->row_ptr = rp; T->col_idx = ci; T->colors = cl;
    return SCC_OK;
}

// Checks a CSR and its colours on the device (Sec. 1.3: a simple undirected
// graph; Sec. 2: colours in [0, k)): EINVAL on any violation.
scc_status validate_csr(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                        const uint8_t *colors, int k, hipStream_t stream, DevMem &mem)
{
    if (n == 0) return nnz == 0 ? SCC_OK : set_error(SCC_EINVAL, "invalid input (an empty graph with nnz = %lld)", (long long)nnz);
    int *err = (int *)mem.get(16);
    if (!err) return set_error(SCC_ENOMEM, "validate");
    int herr = 0;
    hipError_t e = hipMemsetAsync(err, 0, 4, stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_validate_rows, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, stream, row_ptr, n,
                           nnz, err);
        e = hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
    }
    if (e == hipSuccess && herr == 0) {
        GraphView gv{n, row_ptr, col_idx, colors};
        const int64_t m = std::max(n, nnz);
        hipLaunchKernelGGL(k_validate_edges, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, gv, nnz, k, err);
        e = hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
    }
    mem.put(err);
    if (e != hipSuccess) return set_error(SCC_EDEVICE, "validate: %s", hipGetErrorString(e));
    if (herr)
        return set_error(SCC_EINVAL, "invalid input (%s%s%s%s%s%s)", herr & 1 ? "colour >= k " : "",
                         herr & 2 ? "row_ptr not increasing from 0 within [0, nnz] " : "",
                         herr & 4 ? "neighbour out of range or self-loop " : "",
                         herr & 8 ? "row not strictly increasing " : "", herr & 16 ? "asymmetric edge " : "",
                         herr & 32 ? "row_ptr[n] != nnz" : "");
    return SCC_OK;
}

static scc_status validate_graph(scc_table *T)
{
    return validate_csr(T->n, T->nnz_g, T->row_ptr, T->col_idx, T->colors, T->k, T->stream, T->mem);
}

extern "C" scc_status scc_build_table(const scc_csr *g, const uint8_t *colors, int k,
                                      const scc_build_opts *opt, scc_table **out)
{
    if (!out) return set_error(SCC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g || (g->n > 0 && !colors)) return set_error(SCC_EINVAL, "graph or colours NULL");
    if (k < 2 || k > SCC_KMAX) return set_error(SCC_EINVAL, "k = %d not in [2, 8]", k);
    if (g->n < 0 || g->n >= ((int64_t)1 << 31)) return set_error(SCC_EINVAL, "n out of range");
    if (g->nnz < 0 || g->nnz >= ((int64_t)1 << 40) || !g->row_ptr || (g->nnz > 0 && !g->col_idx))
        return set_error(SCC_EINVAL, "bad CSR pointers or size");
    scc_build_opts o{};
    if (opt) o = *opt;
    if (o.rooting != SCC_ROOT_ZERO && o.rooting != SCC_ROOT_ALL && o.rooting != SCC_ROOT_BALANCED)
        return set_error(SCC_EINVAL, "bad rooting");
    if (o.rooting == SCC_ROOT_BALANCED && k < 4) return set_error(SCC_EINVAL, "round skipping needs k >= 4 (k = %d)", k);
    if (o.max_bits == 0) o.max_bits = 128;
    if (o.max_bits != 64 && o.max_bits != 128) return set_error(SCC_EINVAL, "max_bits must be 64 or 128");
    if (o.gather_mode < SCC_GATHER_AUTO || o.gather_mode > SCC_GATHER_ROW)
        return set_error(SCC_EINVAL, "bad gather_mode %d", o.gather_mode);
    if (o.width_test < SCC_WIDTH_AUTO || o.width_test > SCC_WIDTH_PER_WAVE)
        return set_error(SCC_EINVAL, "bad width_test %d", o.width_test);

    scc_table *T = new_table(g, colors, k, o);
    T->gather_mode = o.gather_mode;
    T->width_test = o.width_test;
    scc_status s = attach_graph(T, g, colors);
    if (!s && !o.no_validate) s = validate_graph(T);
    if (!s) s = make_key_maps(T);
    if (!s) s = build_levels(T);
    if (!s) s = build_totals(T);
    if (!s) T->lev[1].nnz = T->n;
    if (!s && o.vlc) s = compact_levels(T);
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

extern "C" scc_status scc_gather_bytes(const scc_table *t, double out[9])
{
    if (!t || !out) return set_error(SCC_EINVAL, "NULL argument");
    scc_status s = gather_stats(const_cast<scc_table *>(t));
    if (s) return s;
    for (int h = 0; h < 9; h++) out[h] = h <= t->k ? t->gather_bytes[h] : 0.0;
    return SCC_OK;
}

extern "C" scc_status scc_combine_bytes(const scc_table *t, double out[9], double *totals)
{
    if (!t || !out || !totals) return set_error(SCC_EINVAL, "NULL argument");
    if (t->vlc) return set_error(SCC_EUNSUPPORTED, "byte counts of tables in the variable-length layout");
    scc_status s = gather_stats(const_cast<scc_table *>(t));
    if (s) return s;
    for (int h = 0; h < 9; h++) out[h] = h <= t->k ? t->combine_bytes[h] : 0.0;
    *totals = t->totals_bytes;
    return SCC_OK;
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
        out->combine_ms[h] = t->combine_ms[h];
        for (int r = 0; r < 3; r++) out->wide_input_rows[h][r] = t->wide_input_rows[h][r];
    }
    out->lane_width_test = t->lane_width_test;
    out->sorted_sum_rows = t->sorted_sum_rows;
    out->grouped_combine = t->grouped_combine;
    out->num_hubs = t->nhub;
    out->bytes = t->bytes;
    out->t[0] = lo64(t->t); out->t[1] = hi64(t->t);
    for (int j = 0; j < t->hlut.num_unr; j++) { out->tj[j][0] = lo64(t->tj[j]); out->tj[j][1] = hi64(t->tj[j]); }
    out->stars[0] = lo64(t->stars); out->stars[1] = hi64(t->stars);
    for (int h = 2; h <= t->k; h++) out->record_bytes += (int64_t)t->lev[h].pool_words * 8;
    out->vlc = t->vlc ? 1 : 0;
    out->totals_ms = t->totals_ms;
    return SCC_OK;
}

// ===========================================================================
// Batched build: many instances (graph x colouring x k) in one persistent
// launch. Work items are (instance, level, phase, vertex tile) in a
// topological order; a resident grid takes them with an in-order ticket
// counter, and an item waits until the items it depends on have completed
// (a per-(instance, level, phase) completion counter). Every item waits only
// on items with smaller tickets, which are held by running workers that never
// wait on later items, so the launch always drains. Inside the launch each
// level's records live in fixed-capacity per-vertex slots; afterwards every
// instance is packed into a standard table.
// ===========================================================================
namespace {

enum { BI_G1 = 0, BI_COMBINE = 1, BI_GATHER = 2, BI_HUB = 3 };

struct BItem {
    int32_t inst;
    int16_t h;
    int16_t phase;
    int32_t dep;      // completion counter waited on, -1 for none
    int32_t need;     // count it must reach
    int32_t done;     // counter incremented when this item completes
    int32_t pad;
    int64_t a, b, c;  // vertex range [a, b); hub chunk: vertex a, edges [b, c)
};

struct BInst {
    GraphView g;
    int k;
    uint64_t *S1;
    u128 *M1;
    GatherArgs G[SCC_KMAX + 1];    // neighbour sums of level h (2..k-1)
    CombineArgs C[SCC_KMAX + 1];   // counts of level h (2..k)
};

struct BatchArgs {
    const BItem *__restrict__ items;
    int64_t nitems;
    const BInst *__restrict__ inst;
    int *counters;
    unsigned long long *ticket;
    int *err;                      // [0] overflow bits, [1] waits that hit the time limit, [2] abort flag
    unsigned long long wait_ticks; // limit of one wait in wall-clock ticks
    uint64_t *hi_scratch;          // per worker: high words of X and S for vertices that need 128 bits
    int64_t hi_stride;             // words per worker
};

__device__ inline long long wave_uniform64(unsigned long long x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return (long long)(((uint64_t)hi << 32) | lo);
}

// One wave per worker. Nothing on the loop's control path is confined to one
// lane: the ticket and completion atomics are issued by the whole wave with an
// addend of 1 in lane 0 only, and the dependency poll runs in every lane with
// its value made scalar. A lane-0-only region on each side of the back edge
// could be merged across it by the compiler, giving the loop a divergent latch
// at which lanes drift apart.
__device__ __attribute__((always_inline)) inline void batch_worker(BatchArgs B)
{
    extern __shared__ uint64_t sm[];
    __shared__ unsigned cnt1[SCC_KMAX];
    const int lane = threadIdx.x;
    const unsigned one = lane == 0 ? 1u : 0u;
    for (;;) {
        const long long it = wave_uniform64(atomicAdd(B.ticket, (unsigned long long)one));
        if (it >= B.nitems) break;
        const BItem I = B.items[it];
        int abort = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&B.err[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (I.dep >= 0 && !abort) {
            const unsigned long long t0 = wall_clock64();
            while (__builtin_amdgcn_readfirstlane(
                       __hip_atomic_load(&B.counters[I.dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < I.need) {
                __builtin_amdgcn_s_sleep(2);
                if (wall_clock64() - t0 > B.wait_ticks) {   // never expected: drain instead of waiting on
                    atomicAdd(&B.err[1], (int)one);
                    atomicMax(&B.err[2], 1);
                    abort = 1;
                    break;
                }
            }
        }
        // acquire: the producers' writes are visible from here on
        if (I.dep >= 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (!abort) {
            // the instance blocks do not change during the launch: reading them through
            // the constant address space keeps their fields in scalar registers
            const BInst &P = *(const BInst *)((const __attribute__((address_space(4))) BInst *)B.inst + I.inst);
            switch (I.phase) {
            case BI_G1:
                for (int64_t v0 = I.a; v0 < I.b; v0 += WAVE)
                    for (uint64_t m = gather1_lanes(P.g, P.k, P.S1, P.M1, v0, min(I.b, v0 + WAVE), GATHER1_LANE_DEG); m;
                         m &= m - 1)
                        gather1_vertex(P.g, P.k, P.S1, P.M1, v0 + (__ffsll((long long)m) - 1), cnt1);
                break;
            case BI_COMBINE: {
                // 64 vertices at a time; at level k under zero-rooting only the colour-0
                // ones, the others getting empty records here (one load for 64 vertices
                // instead of one dependent load each)
                const CombineArgs &C = P.C[I.h];
                uint64_t *hi = B.hi_scratch + (size_t)blockIdx.x * B.hi_stride;
                for (int64_t b0 = I.a; b0 < I.b; b0 += WAVE) {
                    const int64_t vv = b0 + lane;
                    bool z = vv < I.b;
                    if (z && C.zero_only) {
                        z = C.g.colors[vv] == 0;
                        if (!z) { C.meta[vv] = 0; C.Nout[vv] = 0; }
                    }
                    for (uint64_t m = __ballot(z); m; m &= m - 1) {
                        combine_vertex_pf<true, SCC_KMAX - 1, true>(C, b0 + (__ffsll((long long)m) - 1), sm, hi,
                                                                    nullptr, nullptr);
                        __syncthreads();
                    }
                }
                break;
            }
            case BI_GATHER: {
                // 64 rows at a time; at level k-1 under zero-rooting only the colour-0 ones
                const GatherArgs &G = P.G[I.h];
                for (int64_t b0 = I.a; b0 < I.b; b0 += WAVE) {
                    const int64_t vv = b0 + lane;
                    const bool z = vv < I.b && (!G.rows_zero || G.g.colors[vv] == 0);
                    for (uint64_t m = __ballot(z); m; m &= m - 1) {
                        gather_vertex<true>(G, b0 + (__ffsll((long long)m) - 1), sm);
                        __syncthreads();
                    }
                }
                break;
            }
            default:
                hub_chunk<true>(P.G[I.h], I.a, I.b, I.c, sm);
                break;
            }
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // this item's writes before its completion count
        atomicAdd(&B.counters[I.done], (int)one);
    }
}

// Two register budgets of the same worker: the compiler's own (about five waves
// per SIMD) and eight waves per SIMD (a few spills); the schedule autotuner times both.
__global__ void __launch_bounds__(WAVE) k_batch(BatchArgs B) { batch_worker(B); }
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(8, 8))) k_batch_w8(BatchArgs B)
{
    batch_worker(B);
}

// vertex bounds of the cost-split items: item q of s covers the vertices whose
// running cost (degree + SPLIT_C0 per vertex) lies in [q total / s, (q + 1) total / s)
constexpr int64_t SPLIT_C0 = 16;

__global__ void k_item_bounds(BItem *items, int64_t nitems, const BInst *inst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nitems) return;
    BItem I = items[i];
    if (I.pad != 1) return;
    const GraphView g = inst[I.inst].g;
    const int64_t e0 = g.row_ptr[0];
    const u128 total = (u128)(g.row_ptr[g.n] - e0 + SPLIT_C0 * g.n);
    const int64_t s = I.b;
    int64_t b[2];
    for (int r = 0; r < 2; r++) {
        const int64_t q = I.a + r;
        if (q <= 0) { b[r] = 0; continue; }
        if (q >= s) { b[r] = g.n; continue; }
        // smallest v with cost(v) * s >= q * total
        const u128 target = (u128)q * total;
        int64_t lo = 0, hi = g.n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            const u128 c = (u128)(g.row_ptr[mid] - e0 + SPLIT_C0 * mid) * (u128)s;
            if (c >= target) hi = mid; else lo = mid + 1;
        }
        b[r] = lo;
    }
    I.a = b[0];
    I.b = b[1];
    I.pad = 0;
    items[i] = I;
}

struct BatchInstHost {
    scc_table *T = nullptr;
    std::vector<int32_t> hubs;           // ascending
    std::vector<int64_t> hub_rows;       // [2 * nhub]
    int32_t *hubs_dev = nullptr;
    // slots per level, carved from one allocation (slab)
    void *slab = nullptr;
    uint16_t *skey[SCC_KMAX + 1] = {};
    uint64_t *slo[SCC_KMAX + 1] = {}, *shi[SCC_KMAX + 1] = {};
    uint32_t *meta[SCC_KMAX + 1] = {};
    u128 *N[SCC_KMAX + 1] = {};
};

// rows above hub_degree in every instance: sorted vertex ids and their row
// bounds, with three waits for the whole batch
scc_status find_hubs_all(std::vector<BatchInstHost> &H, int hub_degree, hipStream_t st, DevMem &mem,
                         std::vector<std::vector<int32_t>> &hv, std::vector<std::vector<int64_t>> &hr)
{
    const int ni = (int)H.size();
    hv.assign(ni, {});
    hr.assign(ni, {});
    std::vector<int32_t *> ids(ni, nullptr);
    int *cnt = (int *)mem.get((size_t)ni * 4 + 64);
    struct Free {
        DevMem &m; std::vector<int32_t *> &a; int *c;
        ~Free() { for (auto *p : a) m.put(p); m.put(c); }
    } fr{mem, ids, cnt};
    if (!cnt) return set_error(SCC_ENOMEM, "hub counts");
    HIP_TRY(hipMemsetAsync(cnt, 0, (size_t)ni * 4, st));
    for (int i = 0; i < ni; i++) {
        scc_table *T = H[i].T;
        if (!T->n) continue;
        ids[i] = (int32_t *)mem.get((size_t)T->n * 4 + 8);
        if (!ids[i]) return set_error(SCC_ENOMEM, "hub list");
        GraphView g{T->n, T->row_ptr, T->col_idx, T->colors};
        hipLaunchKernelGGL(k_hub_list, dim3((unsigned)((T->n + 255) / 256)), dim3(256), 0, st, g, hub_degree, ids[i],
                           cnt + i);
    }
    std::vector<int> nh(ni, 0);
    HIP_TRY(hipMemcpyAsync(nh.data(), cnt, (size_t)ni * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    bool any = false;
    for (int i = 0; i < ni; i++) {
        if (!nh[i]) continue;
        any = true;
        hv[i].resize(nh[i]);
        HIP_TRY(hipMemcpyAsync(hv[i].data(), ids[i], (size_t)nh[i] * 4, hipMemcpyDeviceToHost, st));
    }
    if (!any) return SCC_OK;
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<int64_t *> rows(ni, nullptr);
    struct FreeRows { DevMem &m; std::vector<int64_t *> &a; ~FreeRows() { for (auto *p : a) m.put(p); } } frr{mem, rows};
    for (int i = 0; i < ni; i++) {
        if (!nh[i]) continue;
        std::sort(hv[i].begin(), hv[i].end());
        scc_table *T = H[i].T;
        rows[i] = (int64_t *)mem.get((size_t)nh[i] * 16 + 16);
        if (!rows[i]) return set_error(SCC_ENOMEM, "hub rows");
        HIP_TRY(hipMemcpyAsync(ids[i], hv[i].data(), (size_t)nh[i] * 4, hipMemcpyHostToDevice, st));
        GraphView g{T->n, T->row_ptr, T->col_idx, T->colors};
        hipLaunchKernelGGL(k_hub_rows, dim3((unsigned)((nh[i] + 255) / 256)), dim3(256), 0, st, g, ids[i], nh[i], rows[i]);
        hr[i].resize(2 * (size_t)nh[i]);
        HIP_TRY(hipMemcpyAsync(hr[i].data(), rows[i], (size_t)nh[i] * 16, hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    return SCC_OK;
}

struct TuneKey {
    std::vector<int64_t> sig;
    bool operator<(const TuneKey &o) const { return sig < o.sig; }
};
std::mutex g_tune_mu;
struct TuneVal { int tile, hub, waves; };
std::map<TuneKey, TuneVal> g_tune;

}  // namespace

static scc_table *new_table(const scc_csr *g, const uint8_t *colors, int k, const scc_build_opts &o)
{
    scc_table *T = new scc_table();
    T->k = k; T->rooting = o.rooting; T->max_bits = o.max_bits;
    T->n = g->n; T->nnz_g = g->nnz;
    T->row_ptr = g->row_ptr; T->col_idx = g->col_idx; T->colors = colors;
    T->stream = (hipStream_t)o.stream;
    T->mem.alloc = o.alloc; T->mem.stream = T->stream;
    T->hub_degree = o.hub_degree > 0 ? o.hub_degree : 1024;
    T->hub_chunk = 256;
    build_lut(k, &T->hlut);
    return T;
}

// One persistent launch over all instances, for one (tile, hub) choice.
// Assumes the per-instance storage exists; fills slots and neighbour sums.
static scc_status batch_launch(std::vector<BatchInstHost> &H, int tile, int hub_degree, int waves, hipStream_t st,
                               DevMem &mem, float *ms_out, int64_t *nitems_out, int *grid_out,
                               std::vector<std::vector<int32_t>> &hv, std::vector<std::vector<int64_t>> &hr)
{
    const void *kern = waves == 8 ? (const void *)k_batch_w8 : (const void *)k_batch;
    const int ni = (int)H.size();
    int kmax = 0;
    for (auto &x : H) kmax = std::max(kmax, x.T->k);
    // hubs for this threshold
    {
        scc_status s = find_hubs_all(H, hub_degree, st, mem, hv, hr);
        if (s) return s;
    }
    // counters: per instance, S-ready[h] (h = 1..k-1) and X-ready[h] (h = 2..k)
    auto cS = [&](int i, int h) { return i * 2 * (SCC_KMAX + 1) + h; };
    auto cX = [&](int i, int h) { return i * 2 * (SCC_KMAX + 1) + (SCC_KMAX + 1) + h; };
    // the exact item count first (the list reaches ~10^6 items of 48 bytes, so
    // growing it by doubling would copy it many times over)
    auto ntiles = [&](int i) {
        const int64_t n = H[i].T->n;
        return std::max<int64_t>((n + tile - 1) / tile, std::min<int64_t>(64, (n + 31) / 32));
    };
    size_t nitems_all = 0;
    for (int i = 0; i < ni; i++) {
        const int k = H[i].T->k;
        nitems_all += (size_t)ntiles(i) * (size_t)(1 + (k - 1) + (k - 2));   // level 1, combines, gathers
        for (size_t q = 0; q < hv[i].size(); q++) {
            const int64_t d = hr[i][2 * q + 1] - hr[i][2 * q];
            nitems_all += (size_t)((d + H[i].T->hub_chunk - 1) / H[i].T->hub_chunk) * (size_t)std::max(0, k - 2);
        }
    }
    std::vector<BItem> items;
    items.reserve(nitems_all);
    std::vector<std::vector<int>> nS(ni, std::vector<int>(SCC_KMAX + 1, 0)), nX(ni, std::vector<int>(SCC_KMAX + 1, 0));
    // Each (instance, phase) is cut into nt items: ceil(n / tile), but at least
    // min(64, ceil(n / 32)) so that a small instance still spreads over many
    // workers. Combine items are runs of consecutive vertices (their work hardly
    // depends on the degree); gather items are ranges of equal edge cost, whose
    // vertex bounds k_item_bounds finds on the device.
    auto tiles = [&](int i, int16_t h, int16_t ph, int dep, int need, int done, bool by_cost) {
        const int64_t n = H[i].T->n;
        const int64_t nt = ntiles(i);
        const int64_t per = nt ? (n + nt - 1) / nt : 0;
        for (int64_t q = 0; q < nt; q++) {
            BItem it{};
            it.inst = i; it.h = h; it.phase = ph; it.dep = dep; it.need = need; it.done = done;
            if (by_cost) { it.pad = 1; it.a = q; it.b = nt; }
            else { it.a = std::min<int64_t>(n, q * per); it.b = std::min<int64_t>(n, (q + 1) * per); }
            items.push_back(it);
        }
        return (int)nt;
    };
    for (int i = 0; i < ni; i++) nS[i][1] = tiles(i, 1, BI_G1, -1, 0, cS(i, 1), true);
    for (int h = 2; h <= kmax; h++) {
        for (int i = 0; i < ni; i++)
            if (H[i].T->k >= h) nX[i][h] = tiles(i, (int16_t)h, BI_COMBINE, cS(i, h - 1), nS[i][h - 1], cX(i, h), false);
        for (int i = 0; i < ni; i++) {
            if (H[i].T->k - 1 < h) continue;
            int c = 0;
            for (size_t q = 0; q < hv[i].size(); q++)
                for (int64_t e = hr[i][2 * q]; e < hr[i][2 * q + 1]; e += H[i].T->hub_chunk) {
                    BItem it{};
                    it.inst = i; it.h = (int16_t)h; it.phase = BI_HUB; it.dep = cX(i, h); it.need = nX[i][h];
                    it.done = cS(i, h);
                    it.a = hv[i][q]; it.b = e; it.c = std::min(hr[i][2 * q + 1], e + H[i].T->hub_chunk);
                    items.push_back(it);
                    c++;
                }
            c += tiles(i, (int16_t)h, BI_GATHER, cX(i, h), nX[i][h], cS(i, h), true);
            nS[i][h] = c;
        }
    }
    // per-instance argument blocks
    std::vector<BInst> inst(ni);
    for (int i = 0; i < ni; i++) {
        scc_table *T = H[i].T;
        const DevLut &HL = T->hlut;
        const int k = T->k;
        const bool zero = T->rooting == SCC_ROOT_ZERO;
        BInst &B = inst[i];
        B.g = GraphView{T->n, T->row_ptr, T->col_idx, T->colors};
        B.k = k;
        B.S1 = T->S[1].lo; B.M1 = T->S[1].M;
        auto slot_src = [&](int h) {
            LevelSrc s{};
            s.skey = H[i].skey[h]; s.slo = H[i].slo[h]; s.shi = H[i].shi[h];
            s.meta = H[i].meta[h]; s.N = H[i].N[h]; s.W = HL.W[h];
            return s;
        };
        for (int h = 2; h < k; h++) {
            GatherArgs &G = B.G[h];
            G.g = B.g; G.k = k; G.nkeys = HL.nkeys; G.WS = HL.WS[h]; G.rows_zero = zero && h == k - 1;
            G.key_lo = HL.off[h]; G.key_n = HL.r[h] * HL.bk[h];
            G.hub_degree = hub_degree;
            G.L = slot_src(h); G.M = T->S[h].M; G.key_sidx = T->key_sidx; G.Slo = T->S[h].lo; G.Shi = T->S[h].hi;
            G.err = nullptr;
        }
        for (int h = 2; h <= k; h++) {
            CombineArgs &C = B.C[h];
            C.g = B.g; C.L = T->dlut; C.h = h; C.zero_only = zero && h == k; C.max_bits = T->max_bits;
            C.bal = 0;
            for (int q = 2; q < h; q++) C.lev[q] = slot_src(q);
            for (int q = 1; q < h; q++) { C.Slo[q] = T->S[q].lo; C.Shi[q] = T->S[q].hi; C.M[q] = T->S[q].M; }
            C.key_xidx = T->key_xidx; C.W = HL.W[h];
            C.late_dma = 0;   // the batched worker stages high words itself: nothing is listed
            C.slot_key = H[i].skey[h]; C.slot_lo = H[i].slo[h]; C.slot_hi = H[i].shi[h];
            C.meta = H[i].meta[h]; C.Nout = H[i].N[h];
            C.bm = nullptr;   // k_mpack sets the bitmaps from the keys
            C.BW = 0;
        }
    }
    const size_t ncount = (size_t)ni * 2 * (SCC_KMAX + 1);
    BItem *ditems = (BItem *)mem.get(items.size() * sizeof(BItem) + 64);
    BInst *dinst = (BInst *)mem.get(inst.size() * sizeof(BInst) + 64);
    int *dcnt = (int *)mem.get(ncount * 4 + 64);
    unsigned long long *dtick = (unsigned long long *)mem.get(64);
    int *derr = (int *)mem.get(64);
    struct Free { DevMem &m; void *p[5]; ~Free() { for (void *q : p) m.put(q); } } fr{mem, {ditems, dinst, dcnt, dtick, derr}};
    if (!ditems || !dinst || !dcnt || !dtick || !derr) return set_error(SCC_ENOMEM, "batch work list");
    for (int i = 0; i < ni; i++)
        for (int h = 2; h < H[i].T->k; h++) inst[i].G[h].err = derr;
    for (int i = 0; i < ni; i++)
        for (int h = 2; h <= H[i].T->k; h++) inst[i].C[h].err = derr;
    HIP_TRY(hipMemcpyAsync(ditems, items.data(), items.size() * sizeof(BItem), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dinst, inst.data(), inst.size() * sizeof(BInst), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(dcnt, 0, ncount * 4, st));
    HIP_TRY(hipMemsetAsync(dtick, 0, 8, st));
    HIP_TRY(hipMemsetAsync(derr, 0, 16, st));
    // cleared hub rows (their sums are merged with atomics)
    for (int i = 0; i < ni; i++) {
        if (hv[i].empty()) continue;
        int32_t *dh = (int32_t *)mem.get(hv[i].size() * 4);
        if (!dh) return set_error(SCC_ENOMEM, "hub ids");
        HIP_TRY(hipMemcpyAsync(dh, hv[i].data(), hv[i].size() * 4, hipMemcpyHostToDevice, st));
        for (int h = 2; h < H[i].T->k; h++)
            hipLaunchKernelGGL(k_hub_prepare, dim3((unsigned)hv[i].size()), dim3(WAVE), 0, st, inst[i].G[h], dh);
        mem.put(dh);   // stream-ordered
    }
    // LDS: the largest need over the instances' gathers and combines (low words;
    // a combine's high words go to the worker's global scratch)
    size_t lds = 0;
    int64_t hi_stride = 0;
    for (int i = 0; i < ni; i++) {
        const DevLut &HL = H[i].T->hlut;
        for (int h = 2; h <= H[i].T->k; h++) {
            lds = std::max(lds, (size_t)(HL.xoff[h] + HL.soff[h]) * 8);
            hi_stride = std::max<int64_t>(hi_stride, HL.xoff[h] + HL.soff[h]);
            if (h < H[i].T->k) lds = std::max(lds, gather_lds(HL.WS[h]));
        }
    }
    hi_stride = (hi_stride + 31) & ~(int64_t)31;
    int dev = 0, ncu = 0, per_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WAVE, lds));
    if (per_cu < 1) return set_error(SCC_EUNSUPPORTED, "batched launch does not fit a CU (LDS %zu)", lds);
    const int grid = std::min<int64_t>((int64_t)ncu * per_cu, (int64_t)items.size());
    int wc_khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&wc_khz, hipDeviceAttributeWallClockRate, dev));
    if (wc_khz <= 0) wc_khz = 100000;
    uint64_t *dhi = (uint64_t *)mem.get((size_t)grid * hi_stride * 8 + 64);
    if (!dhi) return set_error(SCC_ENOMEM, "batch high-word scratch");
    struct FreeHi { DevMem &m; void *p; ~FreeHi() { m.put(p); } } frh{mem, dhi};
    hipLaunchKernelGGL(k_item_bounds, dim3((unsigned)((items.size() + 255) / 256)), dim3(256), 0, st, ditems,
                       (int64_t)items.size(), dinst);
    // a dependency wait longer than 10 s means something is wrong: the launch drains and reports it
    BatchArgs BA{ditems, (int64_t)items.size(), dinst, dcnt, dtick, derr, (unsigned long long)wc_khz * 1000ull * 10ull,
                 dhi, hi_stride};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, st));
    if (waves == 8) hipLaunchKernelGGL(k_batch_w8, dim3((unsigned)grid), dim3(WAVE), lds, st, BA);
    else hipLaunchKernelGGL(k_batch, dim3((unsigned)grid), dim3(WAVE), lds, st, BA);
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int herr[4];
    HIP_TRY(hipMemcpy(herr, derr, sizeof herr, hipMemcpyDeviceToHost));
    HIP_TRY(hipGetLastError());
    if (herr[1]) return set_error(SCC_EDEVICE, "batched launch: %d dependency waits hit the spin limit", herr[1]);
    if (herr[0] & 1) return set_error(SCC_EOVERFLOW, "a count needs more than the allowed bits");
    if (herr[0] & 2) return set_error(SCC_EOVERFLOW, "a neighbour sum may exceed 128 bits");
    if (ms_out) *ms_out = ms;
    if (nitems_out) *nitems_out = (int64_t)items.size();
    if (grid_out) *grid_out = grid;
    return SCC_OK;
}

static scc_status batch_persistent(const scc_instance *inst, int n_inst, const scc_build_opts *opt,
                                   const scc_batch_opts *bopt, scc_table **out, scc_batch_report *rep);

// Extra streams per device for the batch scheduler (slot 0: the persistent
// launch, slot 1: a second level-kernel build; created once, default priority,
// not synchronised with the legacy default stream).
static hipStream_t aux_stream(int dev, int slot)
{
    static std::mutex mu;
    static std::map<std::pair<int, int>, hipStream_t> streams;
    std::lock_guard<std::mutex> lk(mu);
    auto it = streams.find({dev, slot});
    if (it != streams.end()) return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    streams[{dev, slot}] = s;
    return s;
}

// The batch scheduler: instances with at least plain_nnz CSR entries are built
// by the level kernels (exactly as scc_build_table builds them), the others
// together in one persistent launch. When there are both, the persistent launch
// runs from a second host thread on a second stream while the level kernels
// run. The level-kernel instances are taken from a shared queue by two host
// threads on two streams when the two largest of them would fit in free device
// memory together at 1 KiB per CSR entry (one build's kernels then cover the
// other's host waits), else by one. Tables built on a scheduler stream are
// handed back on the caller's stream.
extern "C" scc_status scc_build_batch(const scc_instance *inst, int n_inst, const scc_build_opts *opt,
                                      const scc_batch_opts *bopt, scc_table **out, scc_batch_report *rep)
{
    if (!inst || !out || n_inst < 1) return set_error(SCC_EINVAL, "bad batch arguments");
    for (int i = 0; i < n_inst; i++) out[i] = nullptr;
    scc_batch_opts bo{};
    if (bopt) bo = *bopt;
    const int64_t plain_nnz = bo.plain_nnz > 0 ? bo.plain_nnz : (bo.plain_nnz < 0 ? INT64_MAX : ((int64_t)1 << 21));
    std::vector<int> plain, pers;
    for (int i = 0; i < n_inst; i++) (inst[i].g.nnz >= plain_nnz ? plain : pers).push_back(i);
    scc_batch_report R{};
    auto free_out = [&]() {
        for (int i = 0; i < n_inst; i++) {
            scc_table_destroy(out[i]);
            out[i] = nullptr;
        }
    };
    if (opt && opt->rooting == SCC_ROOT_BALANCED)
        return set_error(SCC_EINVAL, "round skipping is not supported by the batched build");
    std::vector<scc_instance> sub;
    for (int i : pers) sub.push_back(inst[i]);
    std::vector<scc_table *> sout(pers.size(), nullptr);
    scc_build_opts popt{};
    if (opt) popt = *opt;
    const hipStream_t caller = (hipStream_t)popt.stream;
    scc_status sp = SCC_OK;
    std::string perr;
    std::thread worker;
    if (!plain.empty() && !pers.empty()) {
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        const hipStream_t aux = aux_stream(dev, 0);
        if (!aux) return set_error(SCC_EDEVICE, "could not create the batch scheduler's stream");
        popt.stream = (void *)aux;
        worker = std::thread([&, dev] {
            if (hipSetDevice(dev) != hipSuccess) {
                sp = SCC_EDEVICE;
                perr = "hipSetDevice failed in the batch scheduler's thread";
                return;
            }
            sp = batch_persistent(sub.data(), (int)sub.size(), &popt, &bo, sout.data(), &R);
            if (sp) perr = scc_last_error();
        });
    }
    auto free_sub = [&]() {
        for (auto &t : sout) {
            scc_table_destroy(t);
            t = nullptr;
        }
    };
    auto t0 = std::chrono::steady_clock::now();
    scc_status s = SCC_OK, s2 = SCC_OK;
    std::string err2;
    std::atomic<size_t> next{0};
    // builds queued level-kernel instances until the queue is empty or one fails
    auto build_plain = [&](hipStream_t st, bool second, scc_status &res, std::string *err) {
        for (size_t q; (q = next.fetch_add(1)) < plain.size();) {
            const int i = plain[q];
            scc_build_opts po{};
            if (opt) po = *opt;
            po.hub_degree = 0;
            po.vlc = 0;
            if (second) po.stream = (void *)st;
            res = scc_build_table(&inst[i].g, inst[i].colors, inst[i].k, &po, &out[i]);
            if (res) {
                if (err) *err = scc_last_error();
                next = plain.size();
                return;
            }
        }
    };
    hipStream_t st2 = nullptr;
    if (plain.size() >= 2) {
        int64_t a = 0, b = 0;   // the two largest level-kernel instances
        for (int i : plain) {
            const int64_t z = inst[i].g.nnz;
            if (z > a) { b = a; a = z; } else if (z > b) b = z;
        }
        size_t fr = 0, tot = 0;
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipMemGetInfo(&fr, &tot) == hipSuccess &&
            (double)fr > 1024.0 * (double)(a + b))
            st2 = aux_stream(dev, 1);
    }
    std::thread plain2;
    if (st2) {
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        plain2 = std::thread([&, dev] {
            if (hipSetDevice(dev) != hipSuccess) {
                s2 = SCC_EDEVICE;
                err2 = "hipSetDevice failed in the batch scheduler's thread";
                next = plain.size();
                return;
            }
            build_plain(st2, true, s2, &err2);
        });
    }
    build_plain(nullptr, false, s, nullptr);
    if (plain2.joinable()) {
        plain2.join();
        if (!s2 && hipStreamSynchronize(st2) != hipSuccess) {
            s2 = SCC_EDEVICE;
            err2 = "synchronising the batch scheduler's second stream";
        }
        for (int i : plain)   // finished on the second stream: hand over to the caller's
            if (out[i] && out[i]->stream == st2) {
                out[i]->stream = caller;
                out[i]->mem.stream = caller;
            }
        if (!s && s2) {
            s = s2;
            set_error(s2, "%s", err2.c_str());
        }
    }
    const double plain_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (worker.joinable()) {
        worker.join();
        for (scc_table *t : sout)
            if (t) {   // finished and synchronised on the second stream: hand over to the caller's
                t->stream = caller;
                t->mem.stream = caller;
            }
    } else if (!s && !pers.empty()) {
        sp = batch_persistent(sub.data(), (int)sub.size(), opt, &bo, sout.data(), &R);
        if (sp) perr = scc_last_error();
    }
    if (s || sp) {
        const std::string msg = s ? std::string(scc_last_error()) : perr;
        free_out();
        free_sub();
        return set_error(s ? s : sp, "%s", msg.c_str());
    }
    for (size_t q = 0; q < pers.size(); q++) out[pers[q]] = sout[q];
    R.plain_instances = (int)plain.size();
    R.plain_ms = plain_ms;
    if (rep) *rep = R;
    return SCC_OK;
}

static scc_status batch_persistent(const scc_instance *inst, int n_inst, const scc_build_opts *opt,
                                   const scc_batch_opts *bopt, scc_table **out, scc_batch_report *rep)
{
    scc_build_opts o{};
    if (opt) o = *opt;
    if (o.max_bits == 0) o.max_bits = 128;
    if (o.rooting == SCC_ROOT_BALANCED) return set_error(SCC_EINVAL, "round skipping is not supported by the batched build");
    if (o.rooting != SCC_ROOT_ZERO && o.rooting != SCC_ROOT_ALL) return set_error(SCC_EINVAL, "bad rooting");
    if (o.max_bits != 64 && o.max_bits != 128) return set_error(SCC_EINVAL, "max_bits must be 64 or 128");
    scc_batch_opts bo{};
    if (bopt) bo = *bopt;
    hipStream_t st = (hipStream_t)o.stream;
    auto t_start = std::chrono::steady_clock::now();
    std::vector<BatchInstHost> H(n_inst);
    auto fail = [&](scc_status s) {
        for (auto &x : H) {
            if (!x.T) continue;
            x.T->mem.put(x.slab);
            delete x.T;
        }
        return s;
    };
    // tables, lookup tables and storage
    for (int i = 0; i < n_inst; i++) {
        const scc_instance &I = inst[i];
        if (I.k < 2 || I.k > SCC_KMAX) return fail(set_error(SCC_EINVAL, "instance %d: k = %d not in [2, 8]", i, I.k));
        if (I.g.n < 0 || I.g.n >= ((int64_t)1 << 31) || !I.g.row_ptr || (I.g.n > 0 && !I.colors))
            return fail(set_error(SCC_EINVAL, "instance %d: bad graph", i));
        if (I.g.nnz < 0 || I.g.nnz >= ((int64_t)1 << 40) || (I.g.nnz > 0 && !I.g.col_idx))
            return fail(set_error(SCC_EINVAL, "instance %d: bad graph", i));
        scc_table *T = new_table(&I.g, I.colors, I.k, o);
        H[i].T = T;
        scc_status s = attach_graph(T, &I.g, I.colors);
        if (!s && !o.no_validate) s = validate_graph(T);
        if (s) return fail(s);
        s = make_key_maps(T);
        if (s) return fail(s);
        const DevLut &HL = T->hlut;
        const int64_t n = T->n;
        // the neighbour sums of every level in one allocation owned by the table, the
        // slots of every level in another (parts on 256-byte boundaries)
        auto part = [](size_t b) { return (b + 255) & ~(size_t)255; };
        size_t sum_bytes = part((size_t)n * (I.k - 1) * 8 + 8) + part((size_t)n * 16 + 16);
        for (int h = 2; h < I.k; h++) sum_bytes += 2 * part((size_t)n * HL.WS[h] * 8 + 8) + part((size_t)n * 16 + 16);
        char *sums = (char *)T->alloc(sum_bytes + 256);
        if (!sums) return fail(set_error(SCC_ENOMEM, "instance %d: sums (%zu bytes)", i, sum_bytes));
        T->S[1].lo = (uint64_t *)sums; sums += part((size_t)n * (I.k - 1) * 8 + 8);
        T->S[1].M = (u128 *)sums; sums += part((size_t)n * 16 + 16);
        for (int h = 2; h < I.k; h++) {
            const size_t sz = part((size_t)n * HL.WS[h] * 8 + 8);
            T->S[h].lo = (uint64_t *)sums; sums += sz;
            T->S[h].hi = (uint64_t *)sums; sums += sz;
            T->S[h].M = (u128 *)sums; sums += part((size_t)n * 16 + 16);
        }
        size_t slab_bytes = 0;
        for (int h = 2; h <= I.k; h++) {
            const size_t w = (size_t)n * HL.W[h];
            slab_bytes += part(w * 2) + 2 * part(w * 8) + part((size_t)n * 4) + part((size_t)n * 16);
        }
        char *slab = (char *)T->mem.get(slab_bytes + 256);
        if (!slab) return fail(set_error(SCC_ENOMEM, "instance %d: slots (%zu bytes)", i, slab_bytes));
        H[i].slab = slab;
        for (int h = 2; h <= I.k; h++) {
            const size_t w = (size_t)n * HL.W[h];
            H[i].skey[h] = (uint16_t *)slab; slab += part(w * 2);
            H[i].slo[h] = (uint64_t *)slab; slab += part(w * 8);
            H[i].shi[h] = (uint64_t *)slab; slab += part(w * 8);
            H[i].meta[h] = (uint32_t *)slab; slab += part((size_t)n * 4);
            H[i].N[h] = (u128 *)slab; slab += part((size_t)n * 16);
        }
    }
    DevMem mem;
    mem.alloc = o.alloc;
    mem.stream = st;
    // schedule: the caller's choice, a cached tuning result, or a timed probe
    TuneKey key;
    for (int i = 0; i < n_inst; i++) { key.sig.push_back(inst[i].g.n); key.sig.push_back(inst[i].g.nnz); key.sig.push_back(inst[i].k); }
    int tile = bo.tile > 0 ? bo.tile : 256, hubd = bo.hub_degree > 0 ? bo.hub_degree : 1024;
    int waves = bo.waves == 8 ? 8 : 0;
    bool tuned = false;
    scc_batch_report R{};
    if (bo.tile <= 0 && bo.hub_degree <= 0 && bo.waves <= 0) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) { tile = it->second.tile; hubd = it->second.hub; waves = it->second.waves; tuned = true; }
    }
    if (bo.autotune && !tuned) {
        const int tiles[] = {128, 256, 512};
        const int hubs[] = {512, 2048};
        const int wv[] = {0, 8};
        float best = 1e30f;
        for (int w : wv)
            for (int t : tiles)
                for (int hd : hubs) {
                    float ms = 0;
                    std::vector<std::vector<int32_t>> hv;
                    std::vector<std::vector<int64_t>> hr;
                    scc_status s = batch_launch(H, t, hd, w, st, mem, &ms, nullptr, nullptr, hv, hr);
                    if (s) return fail(s);
                    if (R.nprobe < 16) {
                        R.probe_tile[R.nprobe] = t; R.probe_hub[R.nprobe] = hd; R.probe_waves[R.nprobe] = w;
                        R.probe_ms[R.nprobe] = ms; R.nprobe++;
                    }
                    if (ms < best) { best = ms; tile = t; hubd = hd; waves = w; }
                }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = {tile, hubd, waves};
        tuned = true;
    }
    auto t_launch = std::chrono::steady_clock::now();
    float ms = 0;
    int64_t nitems = 0;
    int grid = 0;
    std::vector<std::vector<int32_t>> hub_v;
    std::vector<std::vector<int64_t>> hub_r;
    scc_status s = batch_launch(H, tile, hubd, waves, st, mem, &ms, &nitems, &grid, hub_v, hub_r);
    if (s) return fail(s);
    auto t_pack = std::chrono::steady_clock::now();
    // standard tables, every (instance, level) at once: record sizes and running
    // sums, one read of all pool sizes, one allocation per instance for its pools,
    // locators and bitmaps, then the records; then the totals and one read per table
    std::vector<PackJobDev> jobs;
    std::vector<std::pair<int, int>> job_of;   // (instance, level)
    std::vector<void *> pack_scratch;
    struct FreeScratch {
        std::vector<void *> &v; DevMem &m;
        ~FreeScratch() { for (void *p : v) m.put(p); }
    } frs{pack_scratch, mem};
    auto sget = [&](size_t bytes) { void *p = mem.get(bytes); if (p) pack_scratch.push_back(p); return p; };
    int64_t maxn = 0, maxnb = 1;
    for (int i = 0; i < n_inst; i++) {
        scc_table *T = H[i].T;
        const int64_t n = T->n;
        maxn = std::max(maxn, n);
        const int64_t nb = std::max<int64_t>(1, (n + SCAN_TILE - 1) / SCAN_TILE);
        maxnb = std::max(maxnb, nb);
        uint64_t *words = (uint64_t *)sget((size_t)n * 8 * (T->k - 1) + 64);
        uint64_t *bsum = (uint64_t *)sget((size_t)nb * 8 * (T->k - 1) + 64);
        if (!words || !bsum) return fail(set_error(SCC_ENOMEM, "pack scratch"));
        for (int h = 2; h <= T->k; h++) {
            PackJobDev J{};
            J.n = n; J.W = T->hlut.W[h]; J.BW = (J.W + 63) / 64; J.nkeys = T->hlut.nkeys;
            J.meta = H[i].meta[h]; J.words = words + (size_t)n * (h - 2); J.bsum = bsum + (size_t)nb * (h - 2);
            J.skey = H[i].skey[h]; J.slo = H[i].slo[h]; J.shi = H[i].shi[h]; J.N = H[i].N[h];
            J.key_xidx = T->key_xidx; J.colors = T->colors;
            J.stats = (unsigned long long *)T->dsum + 2 * h;
            jobs.push_back(J);
            job_of.push_back({i, h});
        }
    }
    const int nj = (int)jobs.size();
    uint64_t *dtot = (uint64_t *)sget((size_t)nj * 8 + 64);
    PackJobDev *djobs = (PackJobDev *)sget((size_t)nj * sizeof(PackJobDev) + 64);
    if (!dtot || !djobs) return fail(set_error(SCC_ENOMEM, "pack jobs"));
    for (int j = 0; j < nj; j++) jobs[j].total = dtot + j;
    HIP_TRY(hipMemcpyAsync(djobs, jobs.data(), (size_t)nj * sizeof(PackJobDev), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_mpack_sums, dim3((unsigned)maxnb, (unsigned)nj), dim3(SCAN_T), 0, st, djobs);
    hipLaunchKernelGGL(k_mpack_top, dim3((unsigned)nj), dim3(SCAN_T), 0, st, djobs);
    hipLaunchKernelGGL(k_mpack_apply, dim3((unsigned)maxnb, (unsigned)nj), dim3(SCAN_T), 0, st, djobs);
    std::vector<uint64_t> htot(nj);
    HIP_TRY(hipMemcpyAsync(htot.data(), dtot, (size_t)nj * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    {
        int j = 0;
        for (int i = 0; i < n_inst; i++) {
            scc_table *T = H[i].T;
            const int64_t n = T->n;
            size_t pool_w = 0, bm_w = 0;
            for (int h = 2; h <= T->k; h++) {
                pool_w += (size_t)htot[j + h - 2] + 8;
                bm_w += (size_t)n * ((T->hlut.W[h] + 63) / 64);
            }
            uint64_t *pool = (uint64_t *)T->alloc(pool_w * 8 + 64);
            uint64_t *loc = (uint64_t *)T->alloc((size_t)n * 8 * (T->k - 1) + 64);
            uint64_t *bm = (uint64_t *)T->alloc(bm_w * 8 + 64);
            if (!pool || !loc || !bm) return fail(set_error(SCC_ENOMEM, "instance %d pools (%zu words)", i, pool_w));
            size_t po = 0, bo = 0;
            for (int h = 2; h <= T->k; h++, j++) {
                TableLevel &Lv = T->lev[h];
                Lv.pool = pool + po;
                Lv.pool_words = htot[j];
                Lv.loc = loc + (size_t)n * (h - 2);
                Lv.BW = jobs[j].BW;
                Lv.bm = bm + bo;
                po += (size_t)htot[j] + 8;
                bo += (size_t)n * Lv.BW;
                jobs[j].pool = Lv.pool; jobs[j].loc = Lv.loc; jobs[j].bm = Lv.bm;
            }
        }
    }
    HIP_TRY(hipMemcpyAsync(djobs, jobs.data(), (size_t)nj * sizeof(PackJobDev), hipMemcpyHostToDevice, st));
    if (maxn)
        hipLaunchKernelGGL(k_mpack, dim3((unsigned)std::min<int64_t>((maxn + 3) / 4, 2048), (unsigned)nj), dim3(WAVE), 0,
                           st, djobs);
    for (int i = 0; i < n_inst; i++) {   // stream-ordered releases
        H[i].T->mem.put(H[i].slab);
        H[i].slab = nullptr;
        for (int h = 2; h <= H[i].T->k; h++) {
            H[i].skey[h] = nullptr; H[i].slo[h] = nullptr; H[i].shi[h] = nullptr;
            H[i].meta[h] = nullptr; H[i].N[h] = nullptr;
        }
    }
    HIP_TRY(hipGetLastError());
    for (int i = 0; i < n_inst; i++) {
        scc_table *T = H[i].T;
        // hub list of the chosen threshold, for the sampler's running sums
        T->hub_degree = hubd;
        T->nhub = (int)hub_v[i].size();
        T->hub_host = hub_v[i];
        T->hub_rows_host = hub_r[i];
        s = totals_launch(T);
        if (s) return fail(s);
    }
    for (int i = 0; i < n_inst; i++) {
        s = totals_finish(H[i].T);
        if (s) return fail(s);
    }
    auto t_end = std::chrono::steady_clock::now();
    for (int i = 0; i < n_inst; i++) out[i] = H[i].T;
    if (rep) {
        R.tile = tile; R.hub_degree = hubd; R.waves = waves; R.items = nitems; R.grid = grid; R.launch_ms = ms;
        R.tuned = tuned ? 1 : 0;
        R.pack_ms = std::chrono::duration<double, std::milli>(t_end - t_pack).count();
        R.total_ms = std::chrono::duration<double, std::milli>(t_end - t_launch).count();
        R.setup_ms = std::chrono::duration<double, std::milli>(t_launch - t_start).count();
        *rep = R;
    }
    return SCC_OK;
}
