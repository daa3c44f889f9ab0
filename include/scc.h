/*
 * scc.h -- succinct colour coding on one AMD Instinct MI355X (gfx950).
 *
 * C ABI of libscc.so: the build-up phase (the count table of colourful rooted
 * treelets), the colourful-treelet sampler, induced-graphlet classification
 * and adaptive graphlet sampling of Bressan, Leucci and Panconesi, "Faster
 * motif counting via succinct color coding and adaptive sampling".
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns scc_status; 0 (SCC_OK) is success. On any other value
 *   scc_last_error() returns a message for the calling thread. Output buffers
 *   are not modified on error unless stated.
 * - "device pointer" means memory on the GPU the library runs on (for example a
 *   PyTorch CUDA tensor's data_ptr()); "host pointer" means ordinary memory.
 * - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *   Work is enqueued on that stream; calls that return host values
 *   synchronise it.
 * - The graph is a simple undirected graph in CSR form (Sec. 1.3): row_ptr
 *   int64[n+1], col_idx int32[2m]; every row strictly increasing, symmetric,
 *   without self-loops. Colours are uint8[n] with values in [0, k) (Sec. 2).
 * - Colour sets are k-bit masks (bit j = colour j). A coloured rooted treelet
 *   (T, C), |T| = |C| = h, has the key
 *       key = off_h + rank_h(T) * binom(k, h) + colex(C),
 *   where rank_h orders the rooted shapes on h nodes by their DFS bitstring
 *   (Sec. 3.2: '1' away from the root, '0' back, children in descending
 *   lexicographic order), colex(C) is the number of h-subsets of [k] with a
 *   smaller bitmask, and off_h = sum_{h'<h} r_{h'} binom(k, h'). For k = 8
 *   there are 1991 keys, which fit in 11 bits (Sec. 3.3).
 * - Counts are exact unsigned integers up to 128 bits, passed as (lo, hi)
 *   uint64 pairs.
 */
#ifndef SCC_H
#define SCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SCC_OK = 0,
    SCC_EINVAL = -1,       /* bad argument: k not in [2, 8], colour >= k, non-simple,
                              unsorted or asymmetric CSR, n >= 2^31, bad shape id ... */
    SCC_ENOMEM = -2,       /* device allocation failed */
    SCC_EOVERFLOW = -3,    /* a count would need more bits than allowed (max_bits) */
    SCC_EDEVICE = -4,      /* a HIP runtime error */
    SCC_EEMPTY = -5,       /* nothing to sample: the requested total is 0 */
    SCC_EBUSY = -6,        /* server full: request not admitted */
    SCC_EUNSUPPORTED = -7  /* valid request the library does not support */
} scc_status;

enum { SCC_ROOT_ZERO = 0, SCC_ROOT_ALL = 1, SCC_ROOT_BALANCED = 2 };

typedef struct scc_table scc_table;

/* Device allocator hooks. alloc returns device memory of at least `bytes`
   bytes (or NULL); free releases it. Both are called with the build's stream in
   `stream`, on the caller's thread (scc_build_batch may also call them from its
   second thread, with its second stream, while the call runs). free may be called while work that
   uses the block is still queued on that stream: the allocator must hand the
   block out again only in that stream's order (as a stream-ordered caching
   allocator does), or wait for the stream first. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *stream, void *ctx);
    void *ctx;
} scc_allocator;

typedef struct {
    int64_t n;                 /* number of vertices, < 2^31 */
    int64_t nnz;               /* 2m, length of col_idx, < 2^40 */
    const int64_t *row_ptr;    /* n + 1 entries (never NULL, also for n = 0) */
    const int32_t *col_idx;    /* nnz entries */
    int on_device;             /* 1: row_ptr, col_idx and the call's colours are device
                                  pointers, borrowed for the table's lifetime (the caller
                                  keeps them alive and unchanged); 0: host pointers, copied
                                  by the build into device memory the table owns (the
                                  caller may free them when the call returns) */
} scc_csr;

typedef struct {
    int rooting;               /* SCC_ROOT_ZERO (default): level k kept at colour-0
                                  vertices only (zero-rooting, Sec. 3.4);
                                  SCC_ROOT_ALL: at every vertex (Eq. (1) as is);
                                  SCC_ROOT_BALANCED: round skipping (Sec. 3.3, the
                                  balanced decomposition), k >= 4: level k-1 is not
                                  built and level k holds, at every vertex, only the
                                  designated rooting of each non-star unrooted shape
                                  (scc_balanced_rooting); stars are counted in closed
                                  form and sampled directly (scc_sample). Not
                                  supported by scc_build_batch, scc_ags and AGS
                                  sessions of the server (SCC_EINVAL). */
    int max_bits;              /* 64 or 128 (0 = 128): widest count allowed */
    void *stream;              /* hipStream_t for all work of the build */
    const scc_allocator *alloc;/* NULL: hipMalloc / hipFree */
    int hub_degree;            /* gather rows of at least this degree are split over
                                  many workgroups; 0 = library default */
    int no_validate;           /* 0 (default): check the CSR and colours on the device
                                  before anything reads them, SCC_EINVAL on a violation;
                                  nonzero: skip the check (the caller vouches for the
                                  input; a malformed CSR then makes the kernels read
                                  out of bounds) */
    int gather_mode;           /* neighbour-sum gather of the rows below the hub threshold:
                                  SCC_GATHER_AUTO (0) chooses per level from the level's
                                  record sizes; SCC_GATHER_GROUPED: rows of at most 64
                                  neighbours several to a wave; SCC_GATHER_ROW: one
                                  row per wave. Results are identical in every mode. */
    int vlc;                   /* nonzero: after the build, re-encode every stored level
                                  with variable-length counts (Sec. 3.3): per entry a
                                  u16 of key (11 bits) and byte length l (5 bits), the
                                  count in l bytes, a byte-offset checkpoint every 32
                                  entries. The sampler's running sums are built first.
                                  Every query and sample is unchanged, bit for bit. */
    int width_test;            /* how the combine learns which vertices need 128-bit inputs
                                  (levels 4..k): SCC_WIDTH_AUTO (0): one vertex per lane
                                  first at levels where most rows of the top-level neighbour
                                  sums have high words, else inside the per-vertex combine;
                                  SCC_WIDTH_PER_LANE: one vertex per lane at every such
                                  level; SCC_WIDTH_PER_WAVE: always inside the combine.
                                  Results are identical in every mode. */
} scc_build_opts;

enum { SCC_GATHER_AUTO = 0, SCC_GATHER_GROUPED = 1, SCC_GATHER_ROW = 2 };
enum { SCC_WIDTH_AUTO = 0, SCC_WIDTH_PER_LANE = 1, SCC_WIDTH_PER_WAVE = 2 };

/*
 * scc_build_table -- the build-up phase (Sec. 2.1, Eq. (1)).
 *
 * Computes c(T_C, v) for every colourful rooted treelet (T, C) on h <= k nodes
 * and every vertex v: level 1 is c((., {c_v}), v) = 1 and level h >= 2 is
 *   c(T_C, v) = (1/beta_T) sum_{u ~ v} sum_{C' subset C, |C'| = |T'|}
 *               c(T'_{C'}, v) c(T''_{C \ C'}, u),
 * with (T', T'') the canonical decomposition of T (T'' = the first child
 * subtree of the root, T' = the rest) and beta_T the number of root children
 * whose subtree equals T''. Only non-zero counts are stored (Sec. 3.2, "Count
 * tables"); level k is stored at colour-0 vertices (SCC_ROOT_ZERO) or at all
 * vertices (SCC_ROOT_ALL). Then computes the per-vertex level-k totals eta_v,
 * their running sum over vertices, the total t and per-unrooted-shape totals t_j.
 * Under SCC_ROOT_BALANCED, t_j of a non-star shape is its level-k sum divided
 * by the designated rooting's orbit, the star's t_j is 0 and t is the sum of
 * the non-star t_j; the number of uncoloured k-stars is in scc_table_info.stars
 * (SCC_EOVERFLOW if it needs more than 128 bits).
 *
 * g, colors: device pointers borrowed for the lifetime of the table (the
 * sampler and classifier read them) when g->on_device is set, else host
 * pointers that the build copies. colors: uint8[n]. k in [2, 8]. opt may be
 * NULL (defaults). *out receives a library-owned, immutable table; free it
 * with scc_table_destroy. Errors: SCC_EINVAL (k, sizes, colours or CSR: unless
 * opt->no_validate is set, the CSR is checked to be simple, symmetric and
 * sorted with row_ptr[0] = 0 and row_ptr[n] = nnz, and every colour to be below
 * k, before any other kernel reads them), SCC_EOVERFLOW (a count needs more
 * than max_bits bits; detected from a per-vertex bound before anything wraps),
 * SCC_ENOMEM, SCC_EDEVICE. On error *out is NULL.
 */
scc_status scc_build_table(const scc_csr *g, const uint8_t *colors, int k,
                           const scc_build_opts *opt, scc_table **out);

/* Frees the table and its device memory. NULL is allowed. */
void scc_table_destroy(scc_table *t);

typedef struct {
    int64_t n;
    int k;
    int rooting;
    int num_unrooted;          /* unrooted k-treelet shapes (1,1,1,2,3,6,11,23 for k=1..8) */
    int64_t nnz[9];            /* stored non-zero counts per level h = 1..k (nnz[0] unused) */
    int64_t wide_vertices[9];  /* vertices whose level-h counts are stored with 128 bits */
    int64_t bytes;             /* device bytes held by the table */
    uint64_t t[2];             /* total colourful k-treelet copies (lo, hi) */
    uint64_t tj[32][2];        /* per unrooted shape j */
    double level_ms[9];        /* device time of level h (bound, gather, combine, pack) */
    double gather_ms[9];       /* device time of the neighbour-sum gather of level h */
    int num_hubs;              /* rows gathered in chunks (degree above the hub threshold) */
    uint64_t stars[2];         /* SCC_ROOT_BALANCED: uncoloured k-stars of the graph,
                                  sum_v binom(d_v, k-1) (lo, hi); 0 otherwise */
    int64_t record_bytes;      /* bytes of the stored records of levels 2..k */
    int vlc;                   /* records in the variable-length layout */
    double combine_ms[9];      /* device time of the combine of level h (Eq. (1) products,
                                  compaction, packing; scc_build_table only) */
    double totals_ms;          /* device time of the level-k totals and running sums */
    int64_t wide_input_rows[9][3]; /* vertices of level h combined from 128-bit inputs, by
                                  route (scc_build_table only): [0] high words in neighbour
                                  sums of more than the top level h-1 (none in own records),
                                  [1] in the top-level sums only (a launch of its own, with LDS
                                  for that level's high words; levels in lane_width_test only),
                                  [2] in own records */
    int lane_width_test;       /* bit h: level h's width test (64- or 128-bit inputs) ran one
                                  vertex per lane before the combine, as at levels where most
                                  vertices have high words in their top-level neighbour sums */
    int sorted_sum_rows;       /* bit h: the rows of the level-h neighbour sums were sorted into
                                  64- and 128-bit ones (one per lane) before the gather, as where
                                  many rows border a vertex whose level-h sum needs 128 bits */
    int grouped_combine;       /* bit h: level h was combined four vertices per wave (at most
                                  64 outputs per vertex) */
} scc_table_info;

/* Table summary (host struct; no device work). */
scc_status scc_table_info_get(const scc_table *t, scc_table_info *out);

/*
 * scc_gather_bytes -- algorithmic bytes of each level's neighbour-sum gather
 * (for roofline reports): over the gathered rows v, 4 d_v (neighbour ids) +
 * the neighbours' level-h records (10 B per entry of a 64-bit vertex, 18 B
 * per entry of a 128-bit vertex) + the dense sums written (8 B per entry, 16 B
 * for 128-bit rows). out: host double[9], out[h] for h = 1..k-1. Runs a
 * counting kernel on the table's stream and synchronises it.
 */
scc_status scc_gather_bytes(const scc_table *t, double out[9]);

/*
 * scc_combine_bytes -- algorithmic bytes of each level's combine (Eq. (1) at
 * every vertex that has level h; under zero-rooting level k at colour-0
 * vertices only): the vertex's own records of levels 2..h-1 (10 B per entry,
 * 18 B for a 128-bit vertex; level 1 is implicit), its dense neighbour sums of
 * levels 1..h-1 that were built (8 B per entry, 16 B for rows with high words)
 * and its level-h record written. out: host double[9], out[h] for h = 2..k.
 * *totals: bytes of the level-k totals (the level-k records read; eta_v and
 * its running sum written, 32 B per vertex). Tables in the fixed layout only
 * (SCC_EUNSUPPORTED after a variable-length re-encoding). Runs a counting
 * kernel on the table's stream and synchronises it.
 */
scc_status scc_combine_bytes(const scc_table *t, double out[9], double *totals);

/*
 * scc_occ -- database queries of Sec. 3: occ(T_C, v) (key >= 0: the count of
 * the coloured rooted treelet with that key at v) or occ(v) (key = -1: eta_v,
 * the number of colourful k-treelet copies stored at v; under SCC_ROOT_BALANCED
 * the designated rootings at v, level k-1 being empty). out: host uint64[2]
 * (lo, hi). Errors: SCC_EINVAL for v or key out of range.
 */
scc_status scc_occ(const scc_table *t, int64_t v, int32_t key, uint64_t out[2]);

/*
 * scc_export_level -- the stored level-h records in vertex order: the
 * non-zero counts c(T_C, v) of the coloured rooted treelets on h nodes at each
 * vertex, sorted by key, as the count tables of Sec. 3.2 keep them (pairs of
 * treelet and count, zeros dropped). Level 1 is one count of 1 per vertex, at
 * the key of ({root}, {c_v}).
 * With off == NULL only *nnz_out is set (the number of stored counts).
 * Otherwise off: device int64[n+1] (record of v is [off[v], off[v+1])),
 * key: device uint16[nnz] (ascending within a record), lo/hi: device
 * uint64[nnz] (the count's low and high 64 bits). All caller-owned.
 * Errors: SCC_EINVAL (h outside [1, k]), SCC_ENOMEM (n * 8 bytes of scratch),
 * SCC_EDEVICE. Synchronises `stream`.
 */
scc_status scc_export_level(const scc_table *t, int h, int64_t *nnz_out,
                            int64_t *off, uint16_t *key, uint64_t *lo, uint64_t *hi, void *stream);

/*
 * scc_sample -- colourful k-treelet copies (Sec. 2.2; sample(T) of Sec. 4.1).
 *
 * shape = -1: each colourful k-treelet copy of the graph with probability 1/t;
 * shape = j:  each copy whose unrooted shape is j with probability 1/t_j.
 * Procedure (it fixes the stream, so equal arguments give equal samples):
 * draw X in [0, T) over the admissible level-k counts (vertices ascending, then
 * keys ascending) and take the first (T_C, v) whose running sum exceeds X;
 * then repeatedly decompose (T, C) at x into (T', T''): draw C'' (subsets of
 * C \ {c_x} of size |T''| by ascending bitmask, weight c(T'_{C\C''}, x) *
 * sum_{u~x} c(T''_{C''}, u)), then u ~ x (CSR order, weight c(T''_{C''}, u)),
 * and continue with (T', C \ C'', x) before (T'', C'', u). Uniform integers in
 * [0, N) come from Philox4x64-10 with key (seed, stream_id) and counter
 * (sample index, draw << 32 | attempt, 0, 0), masked to the bit length of N-1
 * and rejected when >= N; draw 0 is the root, draws 1 + 2i and 2 + 2i belong
 * to the i-th decomposition. Sample s uses index first_index + s.
 *
 * Tables built with SCC_ROOT_BALANCED (round skipping, Sec. 3.3): level k
 * holds only designated rootings, so shape = -1 draws the shape first: draw 0
 * picks the non-star shape j with probability t_j / t (first j, ascending,
 * whose running sum of t_j exceeds a uniform integer below t), then shape j is
 * sampled as above with every draw number increased by 1. shape = the star
 * (scc_star_shape) draws an uncoloured k-star of the graph uniformly: the
 * centre v with probability binom(d_v, k-1) / stars (draw 0, running sums over
 * vertices ascending), then k-1 distinct neighbours, the i-th at position r,
 * uniform below d_v - i (draw 1 + i), among the remaining ones, where a taken
 * position is refilled by the last remaining neighbour (CSR positions, a
 * partial Fisher-Yates shuffle); the leaves follow the centre in draw order,
 * each with parent 0.
 *
 * out_verts: device int32[n * k], vertex ids in discovery order, root first.
 * out_parent: device int8[n * k], position of each vertex's parent (-1 for the
 * root). The first call on a table also stores, with the table, the colour of
 * every edge's head in CSR order (one byte per CSR entry), read by the
 * neighbour draw; it changes no sample. Errors: SCC_EINVAL (shape id),
 * SCC_EEMPTY (total 0), SCC_ENOMEM.
 */
scc_status scc_sample(const scc_table *t, int32_t shape, int64_t n, uint64_t seed,
                      uint64_t stream_id, uint64_t first_index,
                      int32_t *out_verts, int8_t *out_parent, void *stream);

/*
 * scc_sample_noalloc -- scc_sample for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation). Same arguments, samples and errors as scc_sample, bit
 * for bit; it calls no hipMalloc, hipFree or allocating routine. Its only
 * scratch, the call's error flags, lives in a static device array of 256
 * bytes (the maximum; it does not grow with n) that each GPU keeps until the
 * process ends; the flags are cleared by a kernel at the start of every call.
 * Every call on one GPU shares that GPU's array, so calls that overlap on one
 * GPU race (serialise them, for example on one stream). It draws only from
 * running sums that already exist: SCC_EINVAL when the draw would need one
 * that is not built yet (per-shape root sums, hub sums built lazily, or the
 * shape-first sums of round skipping) -- one scc_sample call with the same
 * shape, or creating a server on the table, builds them. Before such a call it
 * reads neighbour colours from the colour array instead of the per-edge copy;
 * the samples are the same. Synchronises `stream` to read the flags.
 */
scc_status scc_sample_noalloc(const scc_table *t, int32_t shape, int64_t n, uint64_t seed,
                              uint64_t stream_id, uint64_t first_index,
                              int32_t *out_verts, int8_t *out_parent, void *stream);

/*
 * scc_classify -- graphlet classification of samples (Sec. 4.4).
 * For each sample (k vertices of the table's graph), the induced adjacency
 * code  sum_{i<j} [v_i ~ v_j] 2^{idx(i,j)}  (pairs numbered row by row) and the
 * class id of its graphlet: the rank of its canonical code (the minimum code
 * over all k! vertex orders) among the canonical codes of all connected graphs
 * on k vertices (N_k = 1,1,2,6,21,112,853,11117 for k = 1..8).
 * verts: device int32[n * k]. out_code: device uint32[n] or NULL.
 * out_class: device uint32[n]. The first call for a k builds a per-k lookup
 * table on the device (2^(k(k-1)/2) entries; 512 MiB for k = 8) that is kept
 * until scc_release_caches().
 */
scc_status scc_classify(const scc_table *t, const int32_t *verts, int64_t n,
                        uint32_t *out_code, uint32_t *out_class, void *stream);

/*
 * scc_catalog -- the graphlet classes for k (Sec. 4.4 and Sec. 4.1).
 * num_classes receives N_k. If codes != NULL: host uint32[N_k], canonical code
 * of each class (ascending). If sigma != NULL: host int64[N_k], the number of
 * spanning trees sigma_i (Kirchhoff's matrix-tree theorem). If sigma_ij !=
 * NULL: host int64[N_k * num_unrooted], the spanning trees of H_i of unrooted
 * shape j (row-major by class). Computing sigma_ij for k = 8 takes seconds.
 */
scc_status scc_catalog(int k, int64_t *num_classes, uint32_t *codes, int64_t *sigma,
                       int64_t *sigma_ij, void *stream);

/*
 * scc_ags -- adaptive graphlet sampling (Sec. 4.1, Algorithm AGS), in rounds.
 * Round r draws `round_size` samples of one unrooted shape j with sample
 * indices [drawn, drawn + round_size) of (seed, stream_id), classifies them and
 * adds the hits to c_i and round_size to n_j. Start: the shape with the largest
 * t_j (ties: smaller j). After a round, every class the round hit whose count
 * has reached c_i >= cbar is covered (from then on), and if there is any such
 * class the next shape is chosen again:
 *   j* = argmin_{j: t_j > 0} (1/t_j) sum_{i covered} sigma_ij c_i / w_i,
 *   w_i = sum_j n_j sigma_ij / t_j  (double precision, j and i ascending; a
 * score within a relative 2^-40 of the best so far is a tie, and ties go to
 * the smaller j). Stops when every class is covered or the next round would
 * exceed `budget` samples. round_size = 1 is the algorithm as printed: its
 * switch test runs after every sample whose class has reached cbar.
 * Outputs (host): hits int64[N_k]; w double[N_k] (0 for classes never hit;
 * c_i / w_i estimates the colourful count of class i, divide by p_k =
 * scc_colour_set_probability(k, lambda, k, 1) of the colouring's law (k!/k^k
 * for uniform colours) for the count in the graph); n_j int64[num_unrooted];
 * round_shapes int32[budget /
 * round_size] or NULL; *n_rounds.
 */
scc_status scc_ags(const scc_table *t, int64_t cbar, int64_t round_size, int64_t budget,
                   uint64_t seed, uint64_t stream_id, int64_t *hits, double *w, int64_t *n_j,
                   int32_t *round_shapes, int64_t *n_rounds, void *stream);

/*
 * scc_estimate -- graphlet count estimates (Sec. 2.2). A uniform colourful
 * k-treelet copy spans a copy of graphlet class i with probability
 * c_i sigma_i / t (c_i: colourful copies of class i, sigma_i: its spanning
 * trees, t: the table's total), so from uniform samples (w == NULL) of which
 * hits[i] fell in class i out of n_samples,
 *     c_i = t (hits_i / n_samples) / sigma_i;
 * from an AGS run (w = scc_ags's weights), c_i = hits_i / w_i (0 where w_i = 0).
 * The copies in G are g_i = c_i / p_k, p_k the probability that k given
 * vertices are colourful: scc_colour_set_probability(k, lambda, k, 1) for a
 * biased colouring; p_k <= 0 means uniform colours (k!/k^k).
 * hits: host int64[N_k]; w: host double[N_k] or NULL; out_colourful and
 * out_count: host double[N_k], either may be NULL. FP64, classes ascending.
 * Errors: SCC_EINVAL (NULL table or hits, n_samples <= 0 without w).
 */
scc_status scc_estimate(const scc_table *t, const int64_t *hits, const double *w, int64_t n_samples,
                        double p_k, double *out_colourful, double *out_count);

/* Number of unrooted k-treelet shapes (free trees on k nodes), -1 if k is
   outside [1, 8]. Shape ids j in [0, this) order the shapes by the smallest
   DFS bitstring among their rootings. */
int scc_num_unrooted(int k);

/* Round skipping (Sec. 3.3): the designated rooting of unrooted k-shape j, the
   smallest rooted rank (ascending DFS bitstring among the rooted k-shapes)
   whose canonical decomposition splits the tree into two trees of 2..k-2
   nodes. Returns -1 for the k-star, which has no such rooting, for k < 4 and
   for j or k out of range. *orbit (if not NULL) receives the number of nodes
   of a copy at which rooting it gives the designated rooted shape (0 when
   -1 is returned): SCC_ROOT_BALANCED counts every copy that many times. */
int scc_balanced_rooting(int k, int j, int *orbit);

/* Unrooted shape id of the k-star (the tree with one centre and k-1 leaves),
   -1 if k is outside [2, 8]. */
int scc_star_shape(int k);

/*
 * scc_color_biased -- a biased colouring (Sec. 3.5, "Biased coloring"): colour
 * 0 with probability 1 - (k-1) lambda, each colour in [1, k) with probability
 * lambda. lambda is used as L / 2^32 with L = lambda * 2^32 rounded to the
 * nearest integer, 1 <= L < 2^32 and (k-1) L <= 2^32, so the law is exact: the
 * colour of v is read off the low 32 bits r of the first output of
 * Philox4x64-10 with key (seed, stream_id) and counter (v, 0, 1, 0): colour 0
 * while r < 2^32 - (k-1) L, else 1 + (r - (2^32 - (k-1) L)) / L.
 * colors: device uint8[n], caller-owned; enqueued on `stream`.
 * Errors: SCC_EINVAL (k outside [2, 8], n < 0, lambda out of range).
 */
scc_status scc_color_biased(int64_t n, int k, double lambda, uint64_t seed, uint64_t stream_id,
                            uint8_t *colors, void *stream);

/*
 * scc_colour_set_probability -- the probability that a given set of j vertices
 * receives a given colour set C of size j (one vertex per colour): j!/k^j for
 * independent uniform colours (lambda <= 0); under the biased law with
 * parameter lambda (quantised as in scc_color_biased) j! lambda^j when colour
 * 0 is not in C (has_zero = 0) and j! lambda^(j-1) (1 - (k-1) lambda) when it
 * is. With j = k and has_zero = 1 it is p_k, the probability that a k-vertex
 * set is colourful: t / p_k estimates the number of k-treelet copies of G and
 * (c_i / w_i) / p_k the number of copies of graphlet class i (scc_ags).
 * Returns -1 for arguments out of range. Host only.
 */
double scc_colour_set_probability(int k, double lambda, int j, int has_zero);

/*
 * scc_probe_random_reads -- a measurement aid for roofline reports, not part
 * of the method: the device time of n_reads reads of record_bytes bytes each
 * (a multiple of 8 in [8, 256]) at random record-aligned positions of buf,
 * the access pattern of the neighbour-record gather. Read r loads record
 * mix(r + salt) mod (buf_bytes / record_bytes), one 8-byte word per lane of a
 * group of record_bytes / 8 lanes (mix: a 64-bit finaliser of MurmurHash3).
 * buf: device, caller-owned, 8-byte aligned, zero-filled (a loaded word equal
 * to a fixed nonzero constant is stored to sink, which keeps the loads; with
 * zeros it never happens). sink: device uint64, caller-owned.
 * n_reads * record_bytes / 8 <= 2^31. *ms_out: the kernel's duration (HIP
 * events on `stream`, which the call synchronises).
 * Errors: SCC_EINVAL (null pointer, sizes out of range), SCC_EDEVICE.
 */
scc_status scc_probe_random_reads(const void *buf, uint64_t buf_bytes, int record_bytes, int64_t n_reads,
                                  uint64_t salt, uint64_t *sink, void *stream, float *ms_out);

/* One instance of a batched build: a graph (device pointers, as for
   scc_build_table), its colours and its k. */
typedef struct {
    scc_csr g;
    const uint8_t *colors;
    int k;
} scc_instance;

typedef struct {
    int tile;          /* vertices per work item; 0 = tuned or default (256) */
    int hub_degree;    /* rows above this degree are gathered in chunks; 0 = tuned or default (1024) */
    int autotune;      /* nonzero: when no choice is given and none is cached for a batch of the
                          same shape, time candidate (tile, hub_degree, waves) schedules on this
                          batch and keep the fastest for later batches of the same shape */
    int waves;         /* worker register budget: 8 = eight waves per SIMD (a few spills),
                          0 = tuned or the compiler's own (about five waves per SIMD) */
    int64_t plain_nnz; /* instances with at least this many CSR entries are built by the
                          level kernels, one after another, before the persistent launch
                          (which holds the others); 0 = 2^21, negative = none */
} scc_batch_opts;

typedef struct {
    int tile, hub_degree, waves; /* the schedule used */
    int tuned;                 /* 1 when it came from the autotuner (now or cached) */
    int grid;                  /* resident workgroups of the persistent launch */
    int64_t items;             /* work items */
    double launch_ms;          /* device time of the persistent launch */
    double pack_ms;            /* host-observed time of packing and totals */
    double total_ms;           /* launch + pack (excludes setup and tuning) */
    double setup_ms;           /* allocation, lookup tables and tuning probes */
    int nprobe;
    int probe_tile[16], probe_hub[16], probe_waves[16];
    double probe_ms[16];
    int plain_instances;       /* instances built by the level kernels (plain_nnz) */
    double plain_ms;           /* host-observed time of those builds */
} scc_batch_report;

/*
 * scc_build_batch -- the build-up phase (Sec. 2.1, Eq. (1)) of many instances
 * (graphs x colourings x k) in one persistent launch. The multi-threaded
 * build of Sec. 3.4 assigns vertices to a thread pool; here vertex tiles of
 * every instance and level are work items of one resident grid, ordered so
 * that an item only waits for earlier ones. Instances with at least
 * bopt->plain_nnz CSR entries (large enough to fill the GPU alone) are built by
 * the level kernels of scc_build_table instead, on the caller's stream; when
 * there are both kinds the persistent launch runs meanwhile from a second host
 * thread on a library-owned second stream, and its tables are synchronised
 * before the call returns. Each out[i] receives a table equal
 * to what scc_build_table would build for instance i with the same options
 * (bit for bit). opt applies to every instance (rooting, max_bits, stream,
 * allocator; hub_degree and validate are ignored: the schedule decides the
 * former). bopt and rep may be NULL. Errors as for scc_build_table; on error
 * no table is returned.
 */
scc_status scc_build_batch(const scc_instance *inst, int n_inst, const scc_build_opts *opt,
                           const scc_batch_opts *bopt, scc_table **out, scc_batch_report *rep);

/* ------------------------------------------------------------------------
 * Serving. A server keeps tables resident and answers sampling requests: it
 * admits them in submission order while their outputs fit a device-memory
 * budget, and interleaves the samples of all admitted requests into steps of
 * one sampler launch, so that a request arriving while others run starts at
 * the next step (continuous batching). Every sample is fixed by its table,
 * shape and (seed, stream, index) as in scc_sample, so a request's rows are the
 * same alone and inside any mix of requests. AGS sessions run the rounds of
 * adaptive graphlet sampling (Sec. 4.1) as requests; a session's rounds run
 * one after another, each with the shape chosen after the previous rounds,
 * exactly as scc_ags chooses them.
 * ------------------------------------------------------------------------ */
typedef struct scc_server scc_server;

typedef struct {
    const scc_table *const *tables; /* resident tables, borrowed: they must outlive the server */
    int n_tables;
    int64_t hbm_budget;      /* bytes of device memory for the outputs of admitted requests,
                                allocated once at creation (0 = 1 GiB) */
    int max_pending;         /* submitted requests waiting for admission; beyond it
                                scc_server_submit returns EBUSY (0 = 4096) */
    int max_active;          /* admitted requests that run at once (0 = 256) */
    int64_t step_samples;    /* samples per step when many requests share it (0 = 2^18) */
    int64_t chunk;           /* smallest share of a request in one step (0 = 8192) */
    int grid;                /* sampler workgroups (one wave each) per step (0 = 8192) */
    int fifo;                /* nonzero: one whole request per step, in submission order
                                (the plain first-in first-out server, for comparison) */
    double ags_weight;       /* share of a step an AGS round gets relative to a sample
                                request (a session's later rounds wait for it); 0 = 1 */
    void *stream;            /* hipStream_t of the server's work (NULL: its own stream) */
    const scc_allocator *alloc; /* for the budget and the server's buffers (NULL: hipMalloc) */
    double age_tau;          /* > 0: a request's share also grows with its age, by the
                                factor 1 + (seconds since submission) / age_tau, so that
                                long-waiting requests finish first (tail latency); 0: off */
    int64_t small_request;   /* > 0: requests of at most this many samples are small: each
                                step takes the small requests first, whole, then the others in
                                submission order (no shares); 0: shares as above */
    int64_t small_step;      /* with small_request: a step that holds a small request is cut
                                to this many samples (0: step_samples), so that small requests
                                wait for short steps only */
} scc_server_opts;

enum { SCC_REQ_SAMPLE = 0, SCC_REQ_AGS_ROUND = 1 };

typedef struct {
    int kind;                /* SCC_REQ_SAMPLE or SCC_REQ_AGS_ROUND */
    int table;               /* index into scc_server_opts.tables */
    int shape;               /* SAMPLE: -1 uniform, else an unrooted shape id (AGS: the session's) */
    int classify;            /* SAMPLE: nonzero to also return classes (AGS rounds always classify) */
    int session;             /* AGS_ROUND: id from scc_server_ags_open, on the same table */
    int64_t n;               /* samples, >= 1 */
    uint64_t seed, stream_id, first_index; /* SAMPLE: as for scc_sample (AGS: the session's, the
                                             round starting where the previous one ended) */
} scc_request;

typedef struct {
    int64_t id;
    int status;              /* SCC_OK, EDEVICE, or EBUSY for a request dropped at destruction */
    int k, shape;            /* shape the rows were drawn with */
    int64_t n;
    uint64_t first_index;    /* random index of row 0 */
    const int32_t *verts;    /* device, n x k as scc_sample; valid until scc_server_release */
    const int8_t *parent;    /* device, n x k */
    const uint32_t *cls;     /* device, n classes as scc_classify, or NULL */
    double t_submit, t_admit, t_start, t_done; /* seconds since the server was created */
} scc_result;

typedef struct {
    int64_t submitted, completed, rejected, samples, steps;
    int64_t arena_peak, arena_used;   /* bytes of the budget in use: most ever, now */
    double busy_s;           /* host time spent waiting for steps to finish */
    double span_s;           /* first submission to last completion */
    double p50_ms, p99_ms, mean_ms, max_ms; /* latency, submission to completion */
} scc_server_stats;

/* Builds every running sum the tables' samplers need (all shapes), the class
   lookup tables, the budget arena and the step buffers, then starts the
   server's thread. Errors: EINVAL, ENOMEM, EDEVICE, or a table's EEMPTY. */
scc_status scc_server_create(const scc_server_opts *opt, scc_server **out);
/* Opens an AGS session on table `table` with threshold cbar and random stream
   (seed, stream_id); EEMPTY when the table has no colourful k-treelet. */
scc_status scc_server_ags_open(scc_server *s, int table, int64_t cbar, uint64_t seed, uint64_t stream_id,
                               int *session);
/* A session's state after its finished rounds, as scc_ags reports it
   (hits, w and n_j sized as there; up to `cap` round shapes). */
scc_status scc_server_ags_result(scc_server *s, int session, int64_t *hits, double *w, int64_t *n_j,
                                 int32_t *round_shapes, int64_t cap, int64_t *n_rounds);
/* Queues a request. EBUSY: max_pending requests already wait (not queued);
   ENOMEM: its outputs alone exceed the budget; EINVAL; EEMPTY: nothing to sample. */
scc_status scc_server_submit(scc_server *s, const scc_request *req, int64_t *id);
/* Waits up to timeout_s seconds for a request; EBUSY if it has not finished.
   One waiter per request. */
scc_status scc_server_wait(scc_server *s, int64_t id, double timeout_s, scc_result *out);
/* Returns a finished request's outputs to the budget (EBUSY while it runs);
   its result pointers are invalid afterwards. */
scc_status scc_server_release(scc_server *s, int64_t id);
scc_status scc_server_get_stats(scc_server *s, scc_server_stats *out);
/* Stops the server: requests not yet started are dropped (status EBUSY), the
   steps in flight finish, and every buffer of the server is freed. */
void scc_server_destroy(scc_server *s);

/* ------------------------------------------------------------------------ */
/* k up to 16: sparse records keyed by DFS bitstring (Sec. 3.2)             */
/* ------------------------------------------------------------------------ */
typedef struct scc16_table scc16_table;

typedef struct {
    int rooting;               /* SCC_ROOT_ZERO (default): level k at colour-0 vertices
                                  (Sec. 3.4); SCC_ROOT_ALL: at every vertex */
    void *stream;              /* hipStream_t for all work of the build */
    const scc_allocator *alloc;/* NULL: hipMalloc / hipFree */
    int no_validate;           /* as in scc_build_opts */
    int64_t chunk_terms;       /* terms (neighbour entries or Eq. (1) products) formed and
                                  sorted at a time; 0 = 2^26. Results do not depend on it. */
    int max_bits;              /* count width: 128 or 256; 0 (default) = 128, and the
                                  whole build again at 256 when a count needs more bits */
} scc16_build_opts;

typedef struct {
    int64_t n;
    int k;
    int rooting;
    int64_t nnz[17];           /* stored counts of level h (nnz[0] unused) */
    int64_t terms[17];         /* non-zero products of Eq. (1) formed for level h */
    int64_t nbr_terms[17];     /* neighbour entries gathered into the sums of level h */
    int64_t sum_nnz[17];       /* distinct neighbour sums kept for level h */
    int64_t chunks[17];        /* vertex chunks of level h's products */
    int64_t bytes;             /* device bytes of the stored levels */
    int64_t peak_bytes;        /* largest device working set of the build */
    uint64_t t[4];             /* colourful k-treelet copies, four words, least significant first */
    int count_bits;            /* width of the stored counts: 128 or 256 */
    double level_ms[17];       /* device time of level h (products and its sums) */
    double sort_ms[17];        /* of which radix sorting */
    double sort_bytes[17];     /* algorithmic bytes of those sorts: 32 per element and pass
                                  (8 read by the histogram; 12 read and 12 written by the
                                  scatter) */
    double build_ms;           /* the whole build after validation */
} scc16_table_info;

/*
 * scc16_build_table -- the build-up phase (Sec. 2.1, Eq. (1)) for k in
 * [2, 16], with the treelet representation of Sec. 3.2: a rooted treelet on h
 * nodes is its DFS bitstring s_T of 2(h-1) bits ('1' away from the root, '0'
 * back, the root's child words "1 s 0" in descending lexicographic order,
 * first edge at the most significant bit), and a coloured treelet (T, C) the
 * key s_T << 16 | C (C the k-bit colour mask; 46 bits at most). Every vertex
 * keeps only its non-zero counts, sorted by key (the count tables of Sec. 3.2).
 * c(T_C, v) is as in scc_build_table, T'' being T's largest root child
 * subtree. Counts are exact unsigned integers of 128 bits, or of 256 bits when
 * opt->max_bits asks for them or (max_bits = 0) a count needs more than 128
 * bits; a count, product or sum beyond 256 bits gives SCC_EOVERFLOW. The table
 * holds the levels and t; it has no sampler.
 *
 * g, colors: as in scc_build_table (device pointers borrowed, or host
 * pointers copied). opt may be NULL. *out: free with scc16_table_destroy.
 * Errors: SCC_EINVAL (k, rooting, sizes, colours, CSR), SCC_EOVERFLOW,
 * SCC_ENOMEM (also when one vertex alone forms 2^31 or more terms),
 * SCC_EDEVICE. On error *out is NULL.
 */
scc_status scc16_build_table(const scc_csr *g, const uint8_t *colors, int k, const scc16_build_opts *opt,
                             scc16_table **out);
void scc16_table_destroy(scc16_table *t);
scc_status scc16_table_info_get(const scc16_table *t, scc16_table_info *out);

/*
 * scc16_export_level -- level h's records in vertex order (Sec. 3.2, "Count
 * tables"): off device int64[n+1] (the record of v is [off[v], off[v+1])),
 * key device uint64[nnz] (s_T << 16 | C, ascending within a record), words
 * device uint64[nnz * nwords]: each count as nwords (2 or 4) 64-bit words, least
 * significant first. With off == NULL only *nnz_out is set. Caller-owned
 * outputs. Errors: SCC_EINVAL (h outside [1, k]; nwords not 2 or 4, or 2 for a
 * table of 256-bit counts), SCC_EDEVICE. Synchronises `stream`.
 */
scc_status scc16_export_level(const scc16_table *t, int h, int64_t *nnz_out, int64_t *off, uint64_t *key,
                              uint64_t *words, int nwords, void *stream);

/* Frees the per-k class data kept by scc_classify, scc_catalog and AGS (device
   lookup tables, spanning-tree counts). Call only when no classification, AGS
   run or server is in progress. */
void scc_release_caches(void);

/* Thread-local message for the last non-OK status of this thread. */
const char *scc_last_error(void);

/* Library version string. */
const char *scc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SCC_H */
