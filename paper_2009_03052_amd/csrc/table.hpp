// The count table object behind the C ABI.
#pragma once

#include <map>
#include <mutex>

#include "device.hpp"

// the sampler's hub running sums keep one value per HUB_BLOCK neighbours
constexpr int64_t HUB_BLOCK = 64;

struct TableLevel {
    uint64_t *pool = nullptr;   // packed records
    uint64_t pool_words = 0;
    uint64_t *loc = nullptr;    // [n] record locators
    int64_t nnz = 0;
    int64_t wide = 0;
    uint64_t *bm = nullptr;     // [n * BW] presence bitmaps over the dense level layout
    int BW = 0;
    bool vlc = false;           // records in the variable-length layout
};

struct TableSums {
    uint64_t *lo = nullptr;     // [n * WS_h]
    uint64_t *hi = nullptr;     // high words: [hi_rows * WS_h] rows hrow[v], or [n * WS_h] when hrow is null
    int32_t *hrow = nullptr;    // [n] compact high-word row of v (hubs, then rows with M_h(v) >= 2^64), or -1
    int64_t hi_rows = 0;
    u128 *M = nullptr;          // [n] sum over neighbours of N_h
};

struct scc_table {
    int k = 0, rooting = SCC_ROOT_ZERO, max_bits = 128;
    int64_t n = 0, nnz_g = 0;
    const int64_t *row_ptr = nullptr;
    const int32_t *col_idx = nullptr;
    const uint8_t *colors = nullptr;
    hipStream_t stream = nullptr;
    DevMem mem;
    DevLut hlut;
    DevLut *dlut = nullptr;          // device copy of hlut
    int16_t *key_sidx = nullptr;     // [k * nkeys] neighbour-sum index of a key seen from colour c, or -1
    int16_t *key_xidx = nullptr;     // [k * nkeys] own-count index of a key at a colour-c vertex, or -1
    TableLevel lev[SCC_KMAX + 1];
    TableSums S[SCC_KMAX + 1];
    u128 *eta = nullptr;             // [n] admissible level-k total per vertex (all shapes)
    u128 *pre = nullptr;             // [n] inclusive running sum of eta
    u128 t = 0;                      // colourful k-treelet copies
    u128 tj[32] = {0};
    u128 root_total = 0;             // sum of eta (k * t under SCC_ROOT_ALL)
    // round skipping: running sums of the uncoloured k-stars per vertex, their
    // total, and (built on the first uniform sampling call) the device arrays of
    // the shape-first draw: per-shape root running sums and totals t_j
    u128 *star_pre = nullptr;
    u128 stars = 0;
    const u128 **bal_spre = nullptr;
    u128 *bal_stj = nullptr;
    // device summary read once at the end of a build: [2h], [2h+1] = stored entries and
    // 128-bit vertices of level h; then 32 u128 per-shape totals; then the root total
    uint64_t *dsum = nullptr;
    std::map<int, u128 *> pre_shape; // per unrooted shape: running sums, built on demand
    std::map<int, u128> tot_shape;
    std::mutex mu;
    std::vector<void *> owned;       // every device allocation of the table
    double level_ms[SCC_KMAX + 1] = {0};
    double gather_ms[SCC_KMAX + 1] = {0};
    double gather_bytes[SCC_KMAX + 1] = {0};
    double combine_ms[SCC_KMAX + 1] = {0};     // combine, compaction and packing of level h
    double combine_bytes[SCC_KMAX + 1] = {0};
    int64_t wide_input_rows[SCC_KMAX + 1][3] = {};   // 128-bit-input combines of level h, by route
    int lane_width_test = 0;                   // bit h: level h's width test ran one vertex per lane
    int sorted_sum_rows = 0;                   // bit h: the level-h sums' rows were sorted before the gather
    int grouped_combine = 0;                   // bit h: level h combined four vertices per wave
    double totals_ms = 0, totals_bytes = 0;
    int64_t bytes = 0;
    int hub_degree = 1024;           // rows above this degree are gathered in chunks
    int hub_chunk = 256;             // neighbours per chunk
    int gather_mode = SCC_GATHER_AUTO;
    int width_test = SCC_WIDTH_AUTO;
    bool vlc = false;                // levels re-encoded with variable-length counts after the build
    int nhub = 0;
    bool stats_done = false;
    std::vector<int16_t> key_maps_host;   // host copy of key_sidx then key_xidx (source of their uploads)
    std::vector<int32_t> hub_host;   // hub vertices (ascending) and their row bounds
    std::vector<int64_t> hub_rows_host;
    // per-hub running sums over neighbours of every neighbour-sum entry, for the
    // sampler's neighbour draw (built on the first sampling call)
    bool hubpre_ready = false;
    std::mutex hub_mu;
    int hub_count_pre = 0;           // hubs that have running sums
    int64_t hub_prefix_budget = (int64_t)8 << 30;
    int32_t *hub_index = nullptr;    // [n] hub number or -1
    int64_t *hub_poff = nullptr;     // [nhub * (k+1)] word offset of each (hub, level) block
    uint64_t *hub_pre = nullptr;     // the running sums (low words, then high words if wide)
    // colour of each edge's head in CSR order (colors[col_idx[e]]), built with the
    // hub running sums: the neighbour draw reads it with the edge instead of
    // looking the neighbour's colour up at random
    uint8_t *ecol = nullptr;
    // root draw: every ROOT_STRIDE-th running sum, for a two-level search
    u128 *pre_coarse = nullptr;

    void *alloc(size_t bytes_)
    {
        void *p = mem.get(bytes_);
        if (p) {
            owned.push_back(p);
            bytes += (int64_t)bytes_;
        }
        return p;
    }
    void release(void *p, size_t bytes_)
    {
        for (size_t i = 0; i < owned.size(); i++)
            if (owned[i] == p) {
                owned.erase(owned.begin() + i);
                bytes -= (int64_t)bytes_;
                mem.put(p);
                return;
            }
    }
    ~scc_table()
    {
        for (void *p : owned) mem.put(p);
    }
};

// What a sampling call of this shape draws from (shape -1: t; under round
// skipping the star draws from the uncoloured stars); 0 means nothing to sample.
inline u128 sample_weight(const scc_table *T, int shape)
{
    if (shape < 0) return T->t;
    if (T->rooting == SCC_ROOT_BALANCED && shape == T->hlut.star_unr) return T->stars;
    return T->tj[shape];
}

// Every hub's neighbour running sums and every shape's root running sums.
scc_status prepare_all_sampling(scc_table *T);
// Running sums of admissible level-k totals for one unrooted shape (or all, shape < 0).
scc_status table_prefix(scc_table *T, int shape, const u128 **pre, u128 *total);
// Inclusive running sum of n u128 values on the stream (scratch from T's allocator).
scc_status scan_u128(scc_table *T, const u128 *in, u128 *out, int64_t n);
scc_status scan_u64(scc_table *T, const uint64_t *in, uint64_t *out, int64_t n);
scc_status scan_u32(scc_table *T, const uint32_t *in, uint32_t *out, int64_t n);
// admissible level-k totals of one unrooted shape per vertex (enqueued on T's stream)
void launch_eta_shape(scc_table *T, int shape, u128 *eta);
