// Sampling arguments shared by the plain sampler and the serving sampler, and
// the serving-step structures.
#pragma once

#include "table.hpp"

struct SampleArgs {
    GraphView g;
    const DevLut *L;
    int k, shape, zero;
    LevelView lev[SCC_KMAX + 1];          // 2..k
    const uint64_t *Slo[SCC_KMAX + 1];    // neighbour sums 1..k-1
    const uint64_t *Shi[SCC_KMAX + 1];
    const int32_t *Shrow[SCC_KMAX + 1];   // compact high-word rows, or null (one row per vertex)
    const u128 *M[SCC_KMAX + 1];
    const int16_t *key_xidx;              // [k * nkeys] dense own position of a key, or -1
    int nkeys;
    const int32_t *hub_index;             // [n] hub number or -1
    const int64_t *hub_poff;              // [nhub * (k+1)]
    const uint64_t *hub_pre;
    const uint8_t *ecol;                  // [nnz] colour of each edge's head, or null (read colors[])
    const u128 *pre;                      // running sums of admissible level-k totals
    u128 total;
    // 0: the draw above; 1: shape first (round skipping, shape -1): total = t,
    // spre[j] / stj[j] = shape j's root running sums and t_j (0 for the star);
    // 2: uncoloured k-stars, pre / total = their running sums over centres
    int mode;
    const u128 *const *spre;
    const u128 *stj;
    uint64_t seed, stream, first;
    int64_t nsamp;
    int32_t *verts;
    int8_t *par;
    int *err;
};

// one request's share of a serving step: rows [off, off + count) of the request
struct ServeChunk {
    int32_t arg;       // index of the request's arguments in the step's arrays
    int32_t pad;
    int64_t off;
    int64_t count;
};

// classification of one request's rows in a serving step
struct ServeClassArgs {
    GraphView g;
    int k;
    uint32_t nclass;
    const uint16_t *lut;
    const int32_t *verts;          // n x k
    uint32_t *cls;                 // n
    unsigned long long *hist;      // class histogram added to, or null
};

// Arguments for sampling table T (shape -1: uniform, else that unrooted shape).
// Builds the running sums the draw needs on first use (allocations and waits on
// T's stream). The caller sets seed, stream, first, nsamp, verts, par and err.
scc_status prepare_sampling(scc_table *T, int shape, SampleArgs *A);
// Every hub's neighbour running sums and every shape's root running sums, so
// that later sampling allocates nothing.
scc_status prepare_all_sampling(scc_table *T);
// samples of a serving step: `total` rows over nch chunks (cend: inclusive
// running ends of the chunk counts), one wave per row, grid-stride
void launch_serve_sample(const SampleArgs *args, const ServeChunk *ch, const int64_t *cend, int nch, int64_t total,
                         int *err, int grid, hipStream_t st);
void launch_serve_classify(const ServeClassArgs *args, const ServeChunk *ch, const int64_t *cend, int nch,
                           int64_t total, hipStream_t st);
