/*
 * Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * oracle (oracle.c, test infrastructure): every entry point on small seeded
 * graphs, k = 2..8, all three rootings (classification, AGS and estimates up
 * to k = 7: the k = 8 class catalog alone takes minutes under the sanitizers),
 * and the sparse k <= 16 oracle (oracle16.c) for k = 2..12 and both rootings.
 * Exits 0 when every call succeeds and the sanitizers report nothing (they
 * abort on the first finding).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc_table orc_table;
int orc_build(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const uint8_t *colors, int k, int rooting,
              orc_table **out);
void orc_table_free(orc_table *T);
int64_t orc_level_nnz(const orc_table *T, int h);
int orc_export_level(const orc_table *T, int h, int64_t *off, uint16_t *key, uint64_t *lo, uint64_t *hi);
void orc_totals(const orc_table *T, uint64_t t[2], uint64_t *tj);
void orc_eta(const orc_table *T, uint64_t *out);
int orc_star_count(const orc_table *T, uint64_t out[2]);
int orc_occ(const orc_table *T, int64_t v, int key, uint64_t out[2]);
int orc_sample(const orc_table *T, int shape, int64_t nsamp, uint64_t seed, uint64_t stream, uint64_t first,
               int32_t *verts, int8_t *par);
int orc_classify(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, int k, const int32_t *verts,
                 int64_t nsamp, uint32_t *code, int32_t *cls);
int orc_num_classes(int k);
int orc_num_unrooted(int h);
int orc_num_keys(int k);
int orc_ags(const orc_table *T, int64_t cbar, int64_t round_size, int64_t budget, uint64_t seed, uint64_t stream,
            int64_t *hits, double *w, int64_t *nj, int32_t *shapes, int64_t *nrounds);
int orc_estimate(const orc_table *T, const int64_t *hits, const double *w, int64_t n, double pk, double *c,
                 double *g);
int orc_color_biased(int64_t n, int k, uint32_t L, uint64_t seed, uint64_t stream, uint8_t *out);
int orc_check_csr(int64_t n, const int64_t *row_ptr, const int32_t *col_idx);
typedef struct orc16_table orc16_table;
int orc16_build(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const uint8_t *colors, int k, int rooting,
                orc16_table **out);
void orc16_table_free(orc16_table *T);
int64_t orc16_level_nnz(const orc16_table *T, int h);
int orc16_export_level(const orc16_table *T, int h, int64_t *off, uint64_t *key, uint64_t *words);
void orc16_total(const orc16_table *T, uint64_t t[4]);

static uint64_t rng = 88172645463325252ull;
static uint64_t next(void) { rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17; return rng; }

/* a simple random graph plus a hub, as sorted symmetric CSR */
static void make_graph(int n, int m, int hub, int64_t **rp, int32_t **ci)
{
    char *adj = calloc((size_t)n * n, 1);
    for (int e = 0; e < m; e++) {
        int a = (int)(next() % n), b = (int)(next() % n);
        if (a != b) adj[a * n + b] = adj[b * n + a] = 1;
    }
    for (int v = 1; v < hub && v < n; v++) adj[v] = adj[v * n] = 1;
    *rp = malloc(sizeof(int64_t) * (n + 1));
    int64_t nnz = 0;
    for (int v = 0; v < n; v++) for (int u = 0; u < n; u++) nnz += adj[v * n + u];
    *ci = malloc(sizeof(int32_t) * (nnz ? nnz : 1));
    nnz = 0;
    for (int v = 0; v < n; v++) {
        (*rp)[v] = nnz;
        for (int u = 0; u < n; u++) if (adj[v * n + u]) (*ci)[nnz++] = u;
    }
    (*rp)[n] = nnz;
    free(adj);
}

#define CHECK(x) do { int _s = (x); if (_s) { fprintf(stderr, "%s -> %d (line %d)\n", #x, _s, __LINE__); return 1; } } while (0)

int main(void)
{
    for (int k = 2; k <= 8; k++) {
        const int n = k <= 6 ? 40 : 24;
        int64_t *rp; int32_t *ci;
        make_graph(n, 3 * n, n / 2, &rp, &ci);
        CHECK(orc_check_csr(n, rp, ci));
        uint8_t *col = malloc(n);
        for (int v = 0; v < n; v++) col[v] = (uint8_t)(next() % k);
        for (int rooting = 0; rooting <= 2; rooting++) {
            if (rooting == 2 && k < 4) continue;
            orc_table *T = NULL;
            CHECK(orc_build(n, rp, ci, col, k, rooting, &T));
            for (int h = 1; h <= k; h++) {
                int64_t nnz = orc_level_nnz(T, h);
                int64_t *off = malloc(sizeof(int64_t) * (n + 1));
                uint16_t *key = malloc(2 * (nnz + 1));
                uint64_t *lo = malloc(8 * (nnz + 1)), *hi = malloc(8 * (nnz + 1));
                CHECK(orc_export_level(T, h, off, key, lo, hi));
                free(off); free(key); free(lo); free(hi);
            }
            uint64_t t[2], tj[64], one[2];
            orc_totals(T, t, tj);
            uint64_t *eta = malloc(16 * n);
            orc_eta(T, eta);
            free(eta);
            for (int q = 0; q < 50; q++) {
                int key = (int)(next() % (orc_num_keys(k) + 1)) - 1;
                CHECK(orc_occ(T, (int64_t)(next() % n), key, one));
            }
            if (rooting == 2) CHECK(orc_star_count(T, one));
            if (t[0] || t[1]) {
                int32_t verts[64 * 8]; int8_t par[64 * 8]; uint32_t code[64]; int32_t cls[64];
                CHECK(orc_sample(T, -1, 64, 7, 1, 0, verts, par));
                if (k <= 7) CHECK(orc_classify(n, rp, ci, k, verts, 64, code, cls));
                for (int j = 0; j < orc_num_unrooted(k); j++)
                    if (tj[2 * j] || tj[2 * j + 1]) CHECK(orc_sample(T, j, 16, 9, 2, 5, verts, par));
                if (rooting != 2 && k <= 7) {
                    const int s = orc_num_classes(k), ns = orc_num_unrooted(k);
                    int64_t *hits = calloc(s, 8), *nj = calloc(ns, 8), nr = 0;
                    double *w = calloc(s, 8), *c = calloc(s, 8), *g = calloc(s, 8);
                    int32_t shapes[64];
                    CHECK(orc_ags(T, 5, 20, 1000, 3, 0, hits, w, nj, shapes, &nr));
                    CHECK(orc_estimate(T, hits, w, 0, 0.0, c, g));
                    CHECK(orc_estimate(T, hits, NULL, 1000, 0.0, c, g));
                    free(hits); free(nj); free(w); free(c); free(g);
                }
            }
            orc_table_free(T);
        }
        uint8_t *bc = malloc(n);
        CHECK(orc_color_biased(n, k, 1u << 26, 5, 0, bc));
        free(bc); free(col); free(rp); free(ci);
    }
    for (int k = 2; k <= 12; k++) {
        const int n = 18;
        int64_t *rp; int32_t *ci;
        make_graph(n, 2 * n, 5, &rp, &ci);
        uint8_t *col = malloc(n);
        for (int v = 0; v < n; v++) col[v] = (uint8_t)(next() % k);
        for (int rooting = 0; rooting <= 1; rooting++) {
            orc16_table *T = NULL;
            CHECK(orc16_build(n, rp, ci, col, k, rooting, &T));
            for (int h = 1; h <= k; h++) {
                int64_t nnz = orc16_level_nnz(T, h);
                int64_t *off = malloc(sizeof(int64_t) * (n + 1));
                uint64_t *key = malloc(8 * (nnz + 1)), *words = malloc(32 * (nnz + 1));
                CHECK(orc16_export_level(T, h, off, key, words));
                free(off); free(key); free(words);
            }
            uint64_t t[4];
            orc16_total(T, t);
            orc16_table_free(T);
        }
        free(col); free(rp); free(ci);
    }
    printf("oracle checks done\n");
    return 0;
}
