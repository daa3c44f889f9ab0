/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY. A plain, slow, single-threaded CPU
 * implementation of succinct colour coding (Bressan, Leucci, Panconesi,
 * "Faster motif counting via succinct color coding and adaptive sampling").
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file's library. The GPU library shares no code with it.
 *
 * Every count is an exact unsigned 128-bit integer; every add and multiply is
 * checked and an overflow is reported as an error (nothing wraps).
 *
 * Contents, each following the passage named in its comment:
 *   - rooted treelet shapes as DFS bitstrings (Sec. 3.2, "Treelet
 *     representation", and the example figure of a coloured rooted treelet)
 *   - the build-up dynamic program (Sec. 2.1, Eq. (1)), zero-rooting (Sec. 3.4)
 *   - totals and cumulative counts (Sec. 3.2 "Count tables", Sec. 2.2)
 *   - the uniform / shape-restricted colourful treelet sampler (Sec. 2.2,
 *     Sec. 4.1 sample(T)) with a counter-based generator (Philox4x64-10,
 *     Salmon et al., SC'11)
 *   - induced-graphlet classification by a minimum-over-permutations
 *     adjacency code, spanning-tree numbers (Sec. 4.4 "Graphlet manipulations")
 *   - AGS, adaptive graphlet sampling (Sec. 4.1, Algorithm AGS)
 *   - the estimators of colourful and of all graphlet copies (Sec. 2.2)
 *   - round skipping: balanced rootings, direct star sampling (Sec. 3.3)
 *   - biased colourings and the probability of a colour set (Sec. 3.5)
 *
 * Parity status: every function here is pinned by a CPU test (brute force on
 * tiny graphs, closed forms, printed constants, library cross-checks), except
 * the accuracy of AGS estimates on the paper's real graphs, which is
 * "parity unpinned" (the datasets are not available); AGS itself is pinned by
 * its behaviour on the lollipop graph, by replay and by a sample-by-sample
 * transcription of the printed algorithm.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <stdarg.h>

typedef unsigned __int128 u128;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EOVERFLOW = -3, ORC_EEMPTY = -5 };
enum { ORC_ROOT_ZERO = 0, ORC_ROOT_ALL = 1, ORC_ROOT_BALANCED = 2 };

#define KMAX 8
#define MAXSH 128  /* r_8 = 115 rooted shapes on 8 nodes */
#define SLEN 40

static char g_err[512];
static void set_err(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}
const char *orc_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------- */
/* Rooted treelet shapes (Sec. 3.2, "Treelet representation").               */
/* A rooted tree is written as the DFS bitstring of its edge traversals:      */
/* '1' moving away from the root, '0' moving back. Children are visited in     */
/* descending lexicographic order of their own "1 s 0" strings, which makes    */
/* the string canonical. Shapes of one size are ranked by ascending string.    */
/* ------------------------------------------------------------------------- */
static int sh_n[KMAX + 1];                  /* r_h */
static char sh_s[KMAX + 1][MAXSH][SLEN];    /* canonical strings, ascending */
static int sh_hp[KMAX + 1][MAXSH];          /* size of T' (root part)        */
static int sh_a[KMAX + 1][MAXSH];           /* rank of T' among size-h' shapes */
static int sh_b[KMAX + 1][MAXSH];           /* rank of T'' among size-h'' shapes */
static int sh_beta[KMAX + 1][MAXSH];        /* beta_T */
static int sh_unr[KMAX + 1][MAXSH];         /* unrooted class of each rooted shape */
static int unr_n[KMAX + 1];                 /* number of unrooted shapes of size h */
static int unr_minrank[KMAX + 1][MAXSH];    /* smallest rooted rank of each unrooted class */
static int shapes_ready;

typedef struct { int nn; int adj[16][16]; int deg[16]; } tree_t;

static int cmp_desc(const void *x, const void *y) { return -strcmp((const char *)x, (const char *)y); }
static int cmp_asc(const void *x, const void *y) { return strcmp((const char *)x, (const char *)y); }

/* canonical string of the subtree of t hanging at v, entered from parent p */
static void canon_at(const tree_t *t, int v, int p, char *out)
{
    char kids[16][SLEN];
    int nk = 0;
    for (int i = 0; i < t->deg[v]; i++) {
        int w = t->adj[v][i];
        if (w == p) continue;
        char inner[SLEN];
        canon_at(t, w, v, inner);
        snprintf(kids[nk], SLEN, "1%s0", inner);
        nk++;
    }
    qsort(kids, nk, SLEN, cmp_desc);
    out[0] = 0;
    for (int i = 0; i < nk; i++) strcat(out, kids[i]);
}

static void parse_tree(const char *s, tree_t *t)
{
    int stack[16], sp = 0;
    memset(t, 0, sizeof *t);
    t->nn = 1;
    stack[sp++] = 0;
    for (const char *c = s; *c; c++) {
        if (*c == '1') {
            int x = t->nn++, p = stack[sp - 1];
            t->adj[p][t->deg[p]++] = x;
            t->adj[x][t->deg[x]++] = p;
            stack[sp++] = x;
        } else {
            sp--;
        }
    }
}

static int rank_of(int h, const char *s)
{
    for (int i = 0; i < sh_n[h]; i++)
        if (strcmp(sh_s[h][i], s) == 0) return i;
    return -1;
}

static void build_shapes(void)
{
    if (shapes_ready) return;
    sh_n[1] = 1;
    sh_s[1][0][0] = 0;
    for (int h = 2; h <= KMAX; h++) {
        /* every rooted tree on h nodes arises from one on h-1 nodes by adding a leaf */
        int cnt = 0;
        for (int i = 0; i < sh_n[h - 1]; i++) {
            tree_t t;
            parse_tree(sh_s[h - 1][i], &t);
            for (int x = 0; x < t.nn; x++) {
                tree_t u = t;
                int y = u.nn++;
                u.adj[x][u.deg[x]++] = y;
                u.adj[y][u.deg[y]++] = x;
                char s[SLEN];
                canon_at(&u, 0, -1, s);
                int seen = 0;
                for (int j = 0; j < cnt; j++)
                    if (strcmp(sh_s[h][j], s) == 0) { seen = 1; break; }
                if (!seen) strcpy(sh_s[h][cnt++], s);
            }
        }
        qsort(sh_s[h], cnt, SLEN, cmp_asc);
        sh_n[h] = cnt;
    }
    /* canonical decomposition: T'' = first (largest) root child, T' = the rest */
    for (int h = 2; h <= KMAX; h++) {
        for (int r = 0; r < sh_n[h]; r++) {
            const char *s = sh_s[h][r];
            char words[16][SLEN];
            int nw = 0, depth = 0, start = 0;
            for (int i = 0; s[i]; i++) {
                depth += s[i] == '1' ? 1 : -1;
                if (depth == 0) {
                    memcpy(words[nw], s + start, i + 1 - start);
                    words[nw][i + 1 - start] = 0;
                    nw++;
                    start = i + 1;
                }
            }
            char inner[SLEN], rest[SLEN];
            size_t L = strlen(words[0]);
            memcpy(inner, words[0] + 1, L - 2);
            inner[L - 2] = 0;
            rest[0] = 0;
            for (int i = 1; i < nw; i++) strcat(rest, words[i]);
            int beta = 0;
            for (int i = 0; i < nw; i++) beta += strcmp(words[i], words[0]) == 0;
            int hpp = (int)(L / 2);          /* nodes in T'' */
            int hp = h - hpp;
            sh_hp[h][r] = hp;
            sh_a[h][r] = rank_of(hp, rest);
            sh_b[h][r] = rank_of(hpp, inner);
            sh_beta[h][r] = beta;
        }
    }
    /* unrooted classes: the minimum rooted string over all rootings identifies
       the class; classes are numbered by ascending minimum rooted rank */
    for (int h = 1; h <= KMAX; h++) {
        int minr[MAXSH];
        for (int r = 0; r < sh_n[h]; r++) {
            tree_t t;
            parse_tree(sh_s[h][r], &t);
            int best = sh_n[h];
            for (int x = 0; x < t.nn; x++) {
                char s[SLEN];
                canon_at(&t, x, -1, s);
                int q = rank_of(h, s);
                if (q < best) best = q;
            }
            minr[r] = best;
        }
        int nu = 0;
        for (int q = 0; q < sh_n[h]; q++) {
            int used = 0;
            for (int r = 0; r < sh_n[h]; r++) used |= minr[r] == q;
            if (used) unr_minrank[h][nu++] = q;
        }
        unr_n[h] = nu;
        for (int r = 0; r < sh_n[h]; r++)
            for (int j = 0; j < nu; j++)
                if (unr_minrank[h][j] == minr[r]) sh_unr[h][r] = j;
    }
    shapes_ready = 1;
}

/* ------------------------------------------------------------------------- */
/* Round skipping (Sec. 3.3, balanced treelet decomposition). A rooted shape  */
/* is balanced when its canonical decomposition splits it into two trees of   */
/* at least 2 and at most h-2 nodes. Every unrooted h-shape except the star   */
/* has a balanced rooting (root at an end of an edge whose removal leaves two */
/* trees of >= 2 nodes). The designated rooting of an unrooted shape is its   */
/* smallest balanced rooted rank; its orbit is the number of nodes of a copy  */
/* at which the rooting gives that rank, i.e. how often a copy is counted.   */
/* ------------------------------------------------------------------------- */
static int bal_rank[KMAX + 1][MAXSH];    /* per unrooted class, -1 for none */
static int bal_orbit[KMAX + 1][MAXSH];
static int star_class[KMAX + 1];
static int bal_ready;

static void build_balanced(void)
{
    if (bal_ready) return;
    build_shapes();
    for (int h = 1; h <= KMAX; h++) {
        char star[SLEN] = {0};
        for (int i = 0; i < h - 1; i++) strcat(star, "10");
        star_class[h] = sh_unr[h][rank_of(h, star)];
        for (int j = 0; j < unr_n[h]; j++) { bal_rank[h][j] = -1; bal_orbit[h][j] = 0; }
        for (int r = 0; r < sh_n[h]; r++) {
            if (h < 4) continue;
            const int hpp = h - sh_hp[h][r];
            if (hpp < 2 || hpp > h - 2) continue;
            int *b = &bal_rank[h][sh_unr[h][r]];
            if (*b < 0 || r < *b) *b = r;
        }
        for (int j = 0; j < unr_n[h]; j++) {
            if (bal_rank[h][j] < 0) continue;
            tree_t t;
            parse_tree(sh_s[h][bal_rank[h][j]], &t);
            for (int x = 0; x < t.nn; x++) {
                char cs[SLEN];
                canon_at(&t, x, -1, cs);
                bal_orbit[h][j] += rank_of(h, cs) == bal_rank[h][j];
            }
        }
    }
    bal_ready = 1;
}

int orc_balanced_rank(int h, int j) { build_balanced(); return (h >= 1 && h <= KMAX && j >= 0 && j < unr_n[h]) ? bal_rank[h][j] : -1; }
int orc_balanced_orbit(int h, int j) { build_balanced(); return (h >= 1 && h <= KMAX && j >= 0 && j < unr_n[h]) ? bal_orbit[h][j] : 0; }
int orc_star_class(int h) { build_balanced(); return (h >= 2 && h <= KMAX) ? star_class[h] : -1; }

/* shape queries for tests */
int orc_num_shapes(int h) { build_shapes(); return (h >= 1 && h <= KMAX) ? sh_n[h] : -1; }
int orc_shape_string(int h, int r, char *out, int cap)
{
    build_shapes();
    if (h < 1 || h > KMAX || r < 0 || r >= sh_n[h]) return ORC_EINVAL;
    snprintf(out, cap, "%s", sh_s[h][r]);
    return ORC_OK;
}
int orc_shape_decomp(int h, int r, int *hp, int *a, int *b, int *beta)
{
    build_shapes();
    if (h < 2 || h > KMAX || r < 0 || r >= sh_n[h]) return ORC_EINVAL;
    *hp = sh_hp[h][r]; *a = sh_a[h][r]; *b = sh_b[h][r]; *beta = sh_beta[h][r];
    return ORC_OK;
}
int orc_num_unrooted(int h) { build_shapes(); return (h >= 1 && h <= KMAX) ? unr_n[h] : -1; }
int orc_shape_unrooted(int h, int r) { build_shapes(); return sh_unr[h][r]; }

/* ------------------------------------------------------------------------- */
/* Keys. A coloured rooted treelet (T, C) with |T| = |C| = h gets the integer  */
/* key  off_h + rank_h(T) * binom(k, h) + colex(C), where colex(C) counts the  */
/* h-subsets of [k] whose bitmask is smaller. Keys are ordered like the        */
/* concatenated encoding s_T s_C (Sec. 3.2) within one size; off_h puts sizes  */
/* in increasing order. For k = 8 there are 1991 keys (Sec. 3.3, ITE).        */
/* ------------------------------------------------------------------------- */
static int binom(int n, int r)
{
    if (r < 0 || r > n) return 0;
    int v = 1;
    for (int i = 1; i <= r; i++) v = v * (n - r + i) / i;
    return v;
}
static int popc(unsigned x) { return __builtin_popcount(x); }

typedef struct {
    int k;
    int off[KMAX + 2];
    int nkeys;
    int colex[256];
    int mask_of[KMAX + 1][128]; /* colex rank -> mask, per size */
} keyspace;

static void make_keyspace(int k, keyspace *ks)
{
    build_shapes();
    memset(ks, 0, sizeof *ks);
    ks->k = k;
    int cnt[KMAX + 1] = {0};
    for (unsigned m = 0; m < (1u << k); m++) {
        int p = popc(m);
        ks->colex[m] = cnt[p];
        ks->mask_of[p][cnt[p]] = (int)m;
        cnt[p]++;
    }
    ks->off[1] = 0;
    for (int h = 1; h <= k; h++) ks->off[h + 1] = ks->off[h] + sh_n[h] * binom(k, h);
    ks->nkeys = ks->off[k + 1];
}
static int key_of(const keyspace *ks, int h, int rank, unsigned mask)
{
    return ks->off[h] + rank * binom(ks->k, h) + ks->colex[mask];
}
static void key_decode(const keyspace *ks, int key, int *h, int *rank, unsigned *mask)
{
    int hh = 1;
    while (key >= ks->off[hh + 1]) hh++;
    int rel = key - ks->off[hh];
    int b = binom(ks->k, hh);
    *h = hh;
    *rank = rel / b;
    *mask = (unsigned)ks->mask_of[hh][rel % b];
}
int orc_key(int k, int h, int rank, unsigned mask)
{
    keyspace ks;
    make_keyspace(k, &ks);
    return key_of(&ks, h, rank, mask);
}
int orc_num_keys(int k) { keyspace ks; make_keyspace(k, &ks); return ks.nkeys; }

/* ------------------------------------------------------------------------- */
/* The table                                                                 */
/* ------------------------------------------------------------------------- */
typedef struct {
    int k, rooting;
    int64_t n, nnz_g;
    int64_t *row_ptr;
    int32_t *col_idx;
    uint8_t *colors;
    keyspace ks;
    int64_t *off[KMAX + 1];
    uint16_t *key[KMAX + 1];
    u128 *cnt[KMAX + 1];
    int64_t nnz[KMAX + 1];
    u128 *eta;       /* per-vertex level-k totals */
    u128 t;          /* number of colourful k-treelet copies */
    u128 tj[64];     /* per unrooted shape */
} orc_table;

static int add_ck(u128 *acc, u128 x)
{
    return __builtin_add_overflow(*acc, x, acc) ? ORC_EOVERFLOW : ORC_OK;
}
static int madd_ck(u128 *acc, u128 a, u128 b)
{
    u128 p;
    if (__builtin_mul_overflow(a, b, &p)) return ORC_EOVERFLOW;
    return add_ck(acc, p);
}

int orc_check_csr(int64_t n, const int64_t *row_ptr, const int32_t *col_idx)
{
    if (n < 0 || n >= ((int64_t)1 << 31)) { set_err("n out of range"); return ORC_EINVAL; }
    if (row_ptr[0] != 0) { set_err("row_ptr[0] != 0"); return ORC_EINVAL; }
    for (int64_t v = 0; v < n; v++) {
        if (row_ptr[v + 1] < row_ptr[v]) { set_err("row_ptr decreasing"); return ORC_EINVAL; }
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            int32_t u = col_idx[e];
            if (u < 0 || u >= n) { set_err("neighbour out of range"); return ORC_EINVAL; }
            if (u == v) { set_err("self-loop at %lld", (long long)v); return ORC_EINVAL; }
            if (e > row_ptr[v] && col_idx[e - 1] >= u) { set_err("row %lld not strictly sorted", (long long)v); return ORC_EINVAL; }
            /* symmetry: v must appear in u's row */
            int64_t lo = row_ptr[u], hi = row_ptr[u + 1];
            int found = 0;
            while (lo < hi) {
                int64_t mid = (lo + hi) / 2;
                if (col_idx[mid] == v) { found = 1; break; }
                if (col_idx[mid] < v) lo = mid + 1; else hi = mid;
            }
            if (!found) { set_err("asymmetric edge (%lld,%d)", (long long)v, u); return ORC_EINVAL; }
        }
    }
    return ORC_OK;
}

void orc_table_free(orc_table *T)
{
    if (!T) return;
    for (int h = 1; h <= KMAX; h++) { free(T->off[h]); free(T->key[h]); free(T->cnt[h]); }
    free(T->eta); free(T->row_ptr); free(T->col_idx); free(T->colors);
    free(T);
}

/* binary search of key in v's level-h record; 0 if absent */
static u128 lookup(const orc_table *T, int h, int64_t v, int key)
{
    int64_t lo = T->off[h][v], hi = T->off[h][v + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (T->key[h][mid] == key) return T->cnt[h][mid];
        if (T->key[h][mid] < key) lo = mid + 1; else hi = mid;
    }
    return 0;
}

/* growable record arrays for one level */
typedef struct { uint16_t *key; u128 *cnt; int64_t len, cap; } recbuf;
static int rb_push(recbuf *b, int key, u128 c)
{
    if (b->len == b->cap) {
        int64_t nc = b->cap ? b->cap * 2 : 1024;
        uint16_t *nk = realloc(b->key, nc * sizeof *nk);
        if (!nk) return ORC_ENOMEM;
        b->key = nk;
        u128 *ncn = realloc(b->cnt, nc * sizeof *ncn);
        if (!ncn) return ORC_ENOMEM;
        b->cnt = ncn;
        b->cap = nc;
    }
    b->key[b->len] = (uint16_t)key;
    b->cnt[b->len] = c;
    b->len++;
    return ORC_OK;
}

/*
 * The build-up phase (Sec. 2.1). Level 1: c((., {c_v}), v) = 1. Level h >= 2
 * by Eq. (1):
 *   c(T_C, v) = (1/beta_T) sum_{u ~ v} sum_{C' subset C, |C'| = |T'|}
 *               c(T'_{C'}, v) * c(T''_{C \ C'}, u)
 * with the sum over u taken innermost (distributivity), i.e. through the
 * neighbour sums S(T''_{C''}, v) = sum_{u ~ v} c(T''_{C''}, u). Terms where v's
 * colour is not in C' vanish because c(T'_{C'}, v) = 0 then.
 * Level k is kept at colour-0 vertices only (zero-rooting, Sec. 3.4) or at
 * every vertex.
 */
int orc_build(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
              const uint8_t *colors, int k, int rooting, orc_table **out)
{
    *out = NULL;
    if (k < 2 || k > KMAX) { set_err("k must be in [2, 8]"); return ORC_EINVAL; }
    if (rooting != ORC_ROOT_ZERO && rooting != ORC_ROOT_ALL && rooting != ORC_ROOT_BALANCED) { set_err("bad rooting"); return ORC_EINVAL; }
    if (rooting == ORC_ROOT_BALANCED && k < 4) { set_err("round skipping needs k >= 4"); return ORC_EINVAL; }
    build_balanced();
    int st = orc_check_csr(n, row_ptr, col_idx);
    if (st) return st;
    for (int64_t v = 0; v < n; v++)
        if (colors[v] >= k) { set_err("colour >= k at %lld", (long long)v); return ORC_EINVAL; }

    orc_table *T = calloc(1, sizeof *T);
    if (!T) return ORC_ENOMEM;
    T->k = k; T->rooting = rooting; T->n = n; T->nnz_g = row_ptr[n];
    T->row_ptr = malloc((n + 1) * sizeof(int64_t));
    T->col_idx = malloc((row_ptr[n] ? row_ptr[n] : 1) * sizeof(int32_t));
    T->colors = malloc(n ? n : 1);
    memcpy(T->row_ptr, row_ptr, (n + 1) * sizeof(int64_t));
    memcpy(T->col_idx, col_idx, row_ptr[n] * sizeof(int32_t));
    memcpy(T->colors, colors, n);
    make_keyspace(k, &T->ks);
    const keyspace *ks = &T->ks;

    /* level 1 */
    T->off[1] = malloc((n + 1) * sizeof(int64_t));
    T->key[1] = malloc((n ? n : 1) * sizeof(uint16_t));
    T->cnt[1] = malloc((n ? n : 1) * sizeof(u128));
    for (int64_t v = 0; v < n; v++) {
        T->off[1][v] = v;
        T->key[1][v] = (uint16_t)key_of(ks, 1, 0, 1u << colors[v]);
        T->cnt[1][v] = 1;
    }
    T->off[1][n] = n;
    T->nnz[1] = n;

    /* dense scratch over all keys: own counts X and neighbour sums S at v */
    u128 *X = calloc(ks->nkeys, sizeof(u128));
    u128 *S = calloc(ks->nkeys, sizeof(u128));
    int *touched = malloc(ks->nkeys * sizeof(int));
    int ntouched = 0;
    if (!X || !S || !touched) { free(X); free(S); free(touched); orc_table_free(T); return ORC_ENOMEM; }

    for (int h = 2; h <= k; h++) {
        recbuf rb = {0};
        T->off[h] = malloc((n + 1) * sizeof(int64_t));
        /* round skipping: level k-1 is not built; level k holds only the designated
           (balanced) rooting of every non-star shape, at every vertex */
        const int skip = rooting == ORC_ROOT_BALANCED && h == k - 1;
        for (int64_t v = 0; v < n; v++) {
            T->off[h][v] = rb.len;
            if (skip) continue;
            if (h == k && rooting == ORC_ROOT_ZERO && colors[v] != 0) continue;
            unsigned cv = 1u << colors[v];
            /* S(., v) for every size below h, and v's own X(., v) */
            ntouched = 0;
            for (int hh = 1; hh < h; hh++) {
                for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
                    int64_t u = col_idx[e];
                    for (int64_t q = T->off[hh][u]; q < T->off[hh][u + 1]; q++) {
                        int key = T->key[hh][q];
                        if (S[key] == 0) touched[ntouched++] = key;
                        if (add_ck(&S[key], T->cnt[hh][q])) {
                            set_err("overflow in neighbour sum at v=%lld", (long long)v);
                            st = ORC_EOVERFLOW; goto fail;
                        }
                    }
                }
                for (int64_t q = T->off[hh][v]; q < T->off[hh][v + 1]; q++)
                    X[T->key[hh][q]] = T->cnt[hh][q];
            }
            /* Eq. (1) for every shape of size h and every colour set containing c_v */
            int b = binom(k, h);
            for (int r = 0; r < sh_n[h]; r++) {
                if (h == k && rooting == ORC_ROOT_BALANCED && bal_rank[k][sh_unr[k][r]] != r) continue;
                int hp = sh_hp[h][r], hpp = h - hp;
                int a = sh_a[h][r], bb = sh_b[h][r], beta = sh_beta[h][r];
                for (int ci = 0; ci < b; ci++) {
                    unsigned C = (unsigned)ks->mask_of[h][ci];
                    if (!(C & cv)) continue;
                    u128 acc = 0;
                    /* C' ranges over subsets of C containing c_v, of size |T'| */
                    for (unsigned sub = C; ; sub = (sub - 1) & C) {
                        if ((sub & cv) && popc(sub) == hp) {
                            u128 x = X[key_of(ks, hp, a, sub)];
                            u128 s = S[key_of(ks, hpp, bb, C ^ sub)];
                            if (madd_ck(&acc, x, s)) {
                                set_err("overflow in Eq. (1) at v=%lld", (long long)v);
                                st = ORC_EOVERFLOW; goto fail;
                            }
                        }
                        if (sub == 0) break;
                    }
                    if (acc % (u128)beta != 0) {
                        set_err("internal: sum not divisible by beta at v=%lld", (long long)v);
                        st = ORC_EINVAL; goto fail;
                    }
                    u128 val = acc / (u128)beta;
                    if (val) {
                        if (rb_push(&rb, key_of(ks, h, r, C), val)) { st = ORC_ENOMEM; goto fail; }
                    }
                }
            }
            for (int i = 0; i < ntouched; i++) S[touched[i]] = 0;
            for (int hh = 1; hh < h; hh++)
                for (int64_t q = T->off[hh][v]; q < T->off[hh][v + 1]; q++) X[T->key[hh][q]] = 0;
            continue;
        fail:
            free(rb.key); free(rb.cnt); free(X); free(S); free(touched);
            orc_table_free(T);
            return st;
        }
        T->off[h][n] = rb.len;
        T->key[h] = rb.key ? rb.key : malloc(2);
        T->cnt[h] = rb.cnt ? rb.cnt : malloc(16);
        T->nnz[h] = rb.len;
    }
    free(X); free(S); free(touched);

    /* totals: eta_v (Sec. 3.2), t and t_j (Sec. 2.2 / Sec. 4.1) */
    T->eta = calloc(n ? n : 1, sizeof(u128));
    u128 tsum = 0;
    memset(T->tj, 0, sizeof T->tj);
    for (int64_t v = 0; v < n; v++) {
        for (int64_t q = T->off[k][v]; q < T->off[k][v + 1]; q++) {
            int hh, r; unsigned m;
            key_decode(ks, T->key[k][q], &hh, &r, &m);
            if (add_ck(&T->eta[v], T->cnt[k][q]) || add_ck(&T->tj[sh_unr[k][r]], T->cnt[k][q])) {
                set_err("overflow in totals"); orc_table_free(T); return ORC_EOVERFLOW;
            }
        }
        if (add_ck(&tsum, T->eta[v])) { set_err("overflow in totals"); orc_table_free(T); return ORC_EOVERFLOW; }
    }
    if (rooting == ORC_ROOT_ALL) {
        /* every copy is counted once per rooting */
        if (tsum % (u128)k) { set_err("internal: total not divisible by k"); orc_table_free(T); return ORC_EINVAL; }
        tsum /= (u128)k;
        for (int j = 0; j < unr_n[k]; j++) T->tj[j] /= (u128)k;
    }
    if (rooting == ORC_ROOT_BALANCED) {
        /* every copy is counted once per node of its designated root's orbit */
        tsum = 0;
        for (int j = 0; j < unr_n[k]; j++) {
            if (bal_rank[k][j] < 0) continue;
            if (T->tj[j] % (u128)bal_orbit[k][j]) { set_err("internal: shape total not divisible by its orbit"); orc_table_free(T); return ORC_EINVAL; }
            T->tj[j] /= (u128)bal_orbit[k][j];
            tsum += T->tj[j];
        }
    }
    T->t = tsum;
    *out = T;
    return ORC_OK;
}

int64_t orc_level_nnz(const orc_table *T, int h) { return (h >= 1 && h <= T->k) ? T->nnz[h] : -1; }

int orc_export_level(const orc_table *T, int h, int64_t *off, uint16_t *key, uint64_t *lo, uint64_t *hi)
{
    if (h < 1 || h > T->k) return ORC_EINVAL;
    memcpy(off, T->off[h], (T->n + 1) * sizeof(int64_t));
    for (int64_t q = 0; q < T->nnz[h]; q++) {
        key[q] = T->key[h][q];
        lo[q] = (uint64_t)T->cnt[h][q];
        hi[q] = (uint64_t)(T->cnt[h][q] >> 64);
    }
    return ORC_OK;
}

void orc_totals(const orc_table *T, uint64_t t[2], uint64_t *tj /* 2 * num_unrooted */)
{
    t[0] = (uint64_t)T->t; t[1] = (uint64_t)(T->t >> 64);
    for (int j = 0; j < unr_n[T->k]; j++) { tj[2 * j] = (uint64_t)T->tj[j]; tj[2 * j + 1] = (uint64_t)(T->tj[j] >> 64); }
}

void orc_eta(const orc_table *T, uint64_t *out /* 2n */)
{
    for (int64_t v = 0; v < T->n; v++) { out[2 * v] = (uint64_t)T->eta[v]; out[2 * v + 1] = (uint64_t)(T->eta[v] >> 64); }
}

/* number of (uncoloured) k-stars of G: sum over v of binom(d_v, k-1) */
static u128 binom128(int64_t n, int r)
{
    if (n < r) return 0;
    u128 c = 1;
    for (int i = 1; i <= r; i++) c = c * (u128)(n - r + i) / (u128)i;   /* exact at every step */
    return c;
}

int orc_star_count(const orc_table *T, uint64_t out[2])
{
    u128 s = 0;
    for (int64_t v = 0; v < T->n; v++)
        if (add_ck(&s, binom128(T->row_ptr[v + 1] - T->row_ptr[v], T->k - 1))) { set_err("star count overflows"); return ORC_EOVERFLOW; }
    out[0] = (uint64_t)s; out[1] = (uint64_t)(s >> 64);
    return ORC_OK;
}

/* occ(T_C, v) by key, or occ(v) = eta_v with key = -1 (Sec. 3, database operations) */
int orc_occ(const orc_table *T, int64_t v, int key, uint64_t out[2])
{
    if (v < 0 || v >= T->n) return ORC_EINVAL;
    u128 c;
    if (key < 0) c = T->eta[v];
    else {
        if (key >= T->ks.nkeys) return ORC_EINVAL;
        int h, r; unsigned m;
        key_decode(&T->ks, key, &h, &r, &m);
        c = lookup(T, h, v, key);
    }
    out[0] = (uint64_t)c; out[1] = (uint64_t)(c >> 64);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter-based generator */
/* ------------------------------------------------------------------------- */
void orc_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += W0; k1 += W1; }
        u128 p0 = (u128)M0 * c0, p1 = (u128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/*
 * Uniform integer in [0, N): 128 bits from Philox with key (seed, stream) and
 * counter (sample index, draw index << 32 | attempt, 0, 0), masked to the bit
 * length of N-1, rejected when >= N. N = 1 yields 0 without a draw.
 */
static u128 uniform_below(u128 N, uint64_t seed, uint64_t stream, uint64_t idx, uint32_t draw)
{
    if (N <= 1) return 0;
    u128 nm1 = N - 1;
    int bits = 0;
    while (bits < 128 && (nm1 >> bits) != 0) bits++;
    u128 mask = bits == 128 ? ~(u128)0 : (((u128)1 << bits) - 1);
    for (uint32_t att = 0; ; att++) {
        uint64_t ctr[4] = { idx, ((uint64_t)draw << 32) | att, 0, 0 };
        uint64_t key[2] = { seed, stream };
        uint64_t o[4];
        orc_philox4x64(ctr, key, o);
        u128 r = ((u128)o[1] << 64 | o[0]) & mask;
        if (r < N) return r;
    }
}

int orc_uniform_below(uint64_t nlo, uint64_t nhi, uint64_t seed, uint64_t stream, uint64_t idx,
                      uint32_t draw, uint64_t out[2])
{
    u128 r = uniform_below((u128)nhi << 64 | nlo, seed, stream, idx, draw);
    out[0] = (uint64_t)r; out[1] = (uint64_t)(r >> 64);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Biased colouring (Sec. 3.5, "Biased coloring"): colour 0 with probability  */
/* 1 - (k-1) lambda, each colour i in [1, k) with probability lambda. lambda  */
/* is L / 2^32 for an integer L with (k-1) L <= 2^32, so the law is exact: the */
/* colour of v is read off r = the low 32 bits of the first Philox output for */
/* key (seed, stream) and counter (v, 0, 1, 0): colour 0 while               */
/* r < 2^32 - (k-1) L, else 1 + (r - (2^32 - (k-1) L)) / L.                  */
/* ------------------------------------------------------------------------- */
int orc_color_biased(int64_t n, int k, uint32_t L, uint64_t seed, uint64_t stream, uint8_t *out)
{
    if (k < 2 || k > KMAX || n < 0) { set_err("bad n or k"); return ORC_EINVAL; }
    const uint64_t span = (uint64_t)(k - 1) * L;
    if (L == 0 || span > ((uint64_t)1 << 32)) { set_err("lambda out of range"); return ORC_EINVAL; }
    const uint64_t t0 = ((uint64_t)1 << 32) - span;
    for (int64_t v = 0; v < n; v++) {
        uint64_t ctr[4] = { (uint64_t)v, 0, 1, 0 }, key[2] = { seed, stream }, o[4];
        orc_philox4x64(ctr, key, o);
        const uint64_t r = o[0] & 0xffffffffULL;
        out[v] = r < t0 ? 0 : (uint8_t)(1 + (r - t0) / L);
    }
    return ORC_OK;
}

/* Probability that a given j-vertex set receives exactly the colour set C   */
/* (|C| = j, one vertex per colour) under that law: j! lambda^j when 0 is not */
/* in C, j! lambda^(j-1) (1 - (k-1) lambda) when it is. For j = k this is the  */
/* probability that a k-vertex set is colourful (p_k for the estimates).      */
double orc_colour_set_prob(int k, uint32_t L, int j, int has_zero)
{
    const double lam = (double)L / 4294967296.0;
    double p = 1.0;
    for (int i = 2; i <= j; i++) p *= i;
    for (int i = 0; i < (has_zero ? j - 1 : j); i++) p *= lam;
    if (has_zero) p *= 1.0 - (double)(k - 1) * lam;
    return p;
}

/* ------------------------------------------------------------------------- */
/* Sampling (Sec. 2.2 and sample(T) of Sec. 4.1).                            */
/* (1) draw (T_C, v) with probability proportional to c(T_C, v) among level-k */
/*     entries (restricted to rootings of one unrooted shape if requested);   */
/* (2) recursively: decompose T into (T', T''), draw (C'', u) with probability */
/*     proportional to c(T'_{C \ C''}, v) * c(T''_{C''}, u), in two stages:   */
/*     C'' first (weight c(T'_{C\C''}, v) * S(T''_{C''}, v)), then u ~ v with */
/*     weight c(T''_{C''}, u); continue with (T', C\C'', v) and (T'', C'', u).*/
/* Orders: vertices ascending, record entries by ascending key, C'' by        */
/* ascending bitmask, neighbours in CSR order; the first item whose running   */
/* sum exceeds the drawn value is taken. Draw 0 picks the root; the i-th     */
/* decomposition uses draws 1 + 2i (C'') and 2 + 2i (u).                      */
/* ------------------------------------------------------------------------- */
static int admissible(const orc_table *T, int key, int shape)
{
    if (shape < 0) return 1;
    int h, r; unsigned m;
    key_decode(&T->ks, key, &h, &r, &m);
    return sh_unr[T->k][r] == shape;
}

static int is_root(const orc_table *T, int64_t v)
{
    return T->rooting != ORC_ROOT_ZERO || T->colors[v] == 0;
}

/* running sums over vertices of the admissible level-k weight (shape -1: all) */
static int make_pre(const orc_table *T, int shape, u128 **out)
{
    const int k = T->k;
    u128 *pre = malloc((T->n + 1) * sizeof(u128));
    if (!pre) return ORC_ENOMEM;
    pre[0] = 0;
    for (int64_t v = 0; v < T->n; v++) {
        u128 w = 0;
        if (is_root(T, v))
            for (int64_t q = T->off[k][v]; q < T->off[k][v + 1]; q++)
                if (admissible(T, T->key[k][q], shape) && add_ck(&w, T->cnt[k][q])) { free(pre); return ORC_EOVERFLOW; }
        pre[v + 1] = pre[v];
        if (add_ck(&pre[v + 1], w)) { free(pre); set_err("total overflows 128 bits"); return ORC_EOVERFLOW; }
    }
    *out = pre;
    return ORC_OK;
}

/* One sample of the given admissibility (running sums `pre`) into verts/par;
   the root uses draw doff, the i-th decomposition draws doff + 1 + 2i (C'')
   and doff + 2 + 2i (u). */
static int sample_one(const orc_table *T, int shape, const u128 *pre, uint64_t seed, uint64_t stream, uint64_t idx,
                      uint32_t doff, int32_t *verts, int8_t *par)
{
    const int k = T->k;
    const keyspace *ks = &T->ks;
    u128 X = uniform_below(pre[T->n], seed, stream, idx, doff);
    int64_t lo = 0, hi = T->n;   /* first v with pre[v+1] > X */
    while (lo < hi) { int64_t mid = (lo + hi) / 2; if (pre[mid + 1] > X) hi = mid; else lo = mid + 1; }
    int64_t v = lo;
    u128 res = X - pre[v], cum = 0;
    int rkey = -1;
    for (int64_t q = T->off[k][v]; q < T->off[k][v + 1]; q++) {
        if (!admissible(T, T->key[k][q], shape)) continue;
        cum += T->cnt[k][q];
        if (cum > res) { rkey = T->key[k][q]; break; }
    }
    if (rkey < 0) { set_err("internal: root draw fell off the record"); return ORC_EINVAL; }

    int nv = 0;
    verts[nv] = (int32_t)v; par[nv] = -1; nv++;
    struct { int key; int pos; } stack[2 * KMAX];
    int sp = 0;
    stack[sp].key = rkey; stack[sp].pos = 0; sp++;
    int dec = 0;
    while (sp > 0) {
        sp--;
        int key = stack[sp].key, pos = stack[sp].pos;
        int h, r; unsigned C;
        key_decode(ks, key, &h, &r, &C);
        if (h == 1) continue;
        int64_t x = verts[pos];
        unsigned cv = 1u << T->colors[x];
        int hp = sh_hp[h][r], hpp = h - hp, a = sh_a[h][r], b = sh_b[h][r];
        u128 cT = lookup(T, h, x, key);
        u128 Y = uniform_below((u128)sh_beta[h][r] * cT, seed, stream, idx, doff + 1 + 2 * dec);
        /* stage 1: C'' subset of C \ {c_x}, |C''| = |T''|, ascending bitmask */
        unsigned rest = C & ~cv, Cpp = 0;
        u128 run = 0, Spick = 0;
        int found = 0;
        for (unsigned m = 0; m < (1u << k); m++) {
            if ((m & ~rest) || popc(m) != hpp) continue;
            int kpp = key_of(ks, hpp, b, m);
            u128 Ssum = 0;
            for (int64_t e = T->row_ptr[x]; e < T->row_ptr[x + 1]; e++)
                Ssum += lookup(T, hpp, T->col_idx[e], kpp);
            u128 w = lookup(T, hp, x, key_of(ks, hp, a, C ^ m)) * Ssum;
            run += w;
            if (run > Y) { Cpp = m; Spick = Ssum; found = 1; break; }
        }
        if (!found) { set_err("internal: colour-set draw fell off"); return ORC_EINVAL; }
        /* stage 2: neighbour u with weight c(T''_{C''}, u) */
        int kpp = key_of(ks, hpp, b, Cpp);
        u128 Z = uniform_below(Spick, seed, stream, idx, doff + 2 + 2 * dec);
        u128 run2 = 0;
        int64_t u = -1;
        for (int64_t e = T->row_ptr[x]; e < T->row_ptr[x + 1]; e++) {
            run2 += lookup(T, hpp, T->col_idx[e], kpp);
            if (run2 > Z) { u = T->col_idx[e]; break; }
        }
        if (u < 0) { set_err("internal: neighbour draw fell off"); return ORC_EINVAL; }
        int upos = nv;
        verts[nv] = (int32_t)u; par[nv] = (int8_t)pos; nv++;
        dec++;
        stack[sp].key = kpp; stack[sp].pos = upos; sp++;
        stack[sp].key = key_of(ks, hp, a, C ^ Cpp); stack[sp].pos = pos; sp++;
    }
    return ORC_OK;
}

/* Uncoloured k-stars (round skipping, Sec. 3.3): the centre v with probability
   proportional to binom(d_v, k-1) (draw 0), then k-1 distinct neighbours, the
   i-th uniform among those not taken yet (draw 1 + i): position r of the
   remaining d_v - i neighbours, where a taken position is refilled by the last
   remaining one. Leaves come in draw order, each with parent 0. */
static int sample_stars(const orc_table *T, int64_t nsamp, uint64_t seed, uint64_t stream, uint64_t first_index,
                        int32_t *out_verts, int8_t *out_parent)
{
    const int k = T->k;
    u128 *pre = malloc((T->n + 1) * sizeof(u128));
    if (!pre) return ORC_ENOMEM;
    pre[0] = 0;
    for (int64_t v = 0; v < T->n; v++) {
        pre[v + 1] = pre[v];
        if (add_ck(&pre[v + 1], binom128(T->row_ptr[v + 1] - T->row_ptr[v], k - 1))) { free(pre); set_err("star count overflows"); return ORC_EOVERFLOW; }
    }
    if (pre[T->n] == 0) { free(pre); set_err("no k-star to sample"); return ORC_EEMPTY; }
    for (int64_t s = 0; s < nsamp; s++) {
        uint64_t idx = first_index + (uint64_t)s;
        int32_t *verts = out_verts + s * k;
        int8_t *par = out_parent + s * k;
        u128 X = uniform_below(pre[T->n], seed, stream, idx, 0);
        int64_t lo = 0, hi = T->n;
        while (lo < hi) { int64_t mid = (lo + hi) / 2; if (pre[mid + 1] > X) hi = mid; else lo = mid + 1; }
        const int64_t v = lo, d = T->row_ptr[v + 1] - T->row_ptr[v];
        verts[0] = (int32_t)v; par[0] = -1;
        int64_t mpos[KMAX], mval[KMAX];   /* positions refilled so far */
        int nm = 0;
        for (int i = 0; i < k - 1; i++) {
            int64_t r = (int64_t)uniform_below((u128)(d - i), seed, stream, idx, 1 + i);
            int64_t got = r, last = d - 1 - i, lastval = last;
            for (int q = 0; q < nm; q++) { if (mpos[q] == r) got = mval[q]; if (mpos[q] == last) lastval = mval[q]; }
            verts[1 + i] = T->col_idx[T->row_ptr[v] + got];
            par[1 + i] = 0;
            int q = 0;
            while (q < nm && mpos[q] != r) q++;
            if (q == nm) nm++;
            mpos[q] = r; mval[q] = lastval;
        }
    }
    free(pre);
    return ORC_OK;
}

int orc_sample(const orc_table *T, int shape, int64_t nsamp, uint64_t seed, uint64_t stream,
               uint64_t first_index, int32_t *out_verts, int8_t *out_parent)
{
    const int k = T->k;
    if (shape >= unr_n[k]) { set_err("shape id out of range"); return ORC_EINVAL; }
    const int bal = T->rooting == ORC_ROOT_BALANCED;
    if (bal && shape == star_class[k]) return sample_stars(T, nsamp, seed, stream, first_index, out_verts, out_parent);
    /* shape-first under round skipping: draw 0 picks the shape (weight t_j),
       then the shape's sample follows with every draw index shifted by one */
    const int first = bal && shape < 0;
    u128 *pre[MAXSH] = {0};
    int st = ORC_OK;
    if (first) {
        for (int j = 0; j < unr_n[k] && !st; j++)
            if (bal_rank[k][j] >= 0 && T->tj[j] > 0) st = make_pre(T, j, &pre[j]);
    } else {
        st = make_pre(T, shape, &pre[0]);
    }
    if (st) { for (int j = 0; j < MAXSH; j++) free(pre[j]); return st; }
    if ((first && T->t == 0) || (!first && pre[0][T->n] == 0)) {
        for (int j = 0; j < MAXSH; j++) free(pre[j]);
        set_err("no colourful k-treelet to sample");
        return ORC_EEMPTY;
    }
    for (int64_t s = 0; s < nsamp && !st; s++) {
        uint64_t idx = first_index + (uint64_t)s;
        if (first) {
            u128 X = uniform_below(T->t, seed, stream, idx, 0), cum = 0;
            int j = 0;
            for (; j < unr_n[k]; j++) {
                if (bal_rank[k][j] < 0) continue;
                cum += T->tj[j];
                if (cum > X) break;
            }
            st = sample_one(T, j, pre[j], seed, stream, idx, 1, out_verts + s * k, out_parent + s * k);
        } else {
            st = sample_one(T, shape, pre[0], seed, stream, idx, 0, out_verts + s * k, out_parent + s * k);
        }
    }
    for (int j = 0; j < MAXSH; j++) free(pre[j]);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Graphlets (Sec. 4.4). The adjacency code of an ordered vertex tuple is     */
/* sum_{i<j} adj(i,j) 2^{idx(i,j)} with pairs (i,j) numbered row by row. The  */
/* canonical code of a graphlet is the minimum code over all k! orderings;    */
/* class ids rank the canonical codes of all connected k-vertex graphs.       */
/* ------------------------------------------------------------------------- */
static int pair_idx[KMAX][KMAX];
static int pair_i[32], pair_j[32];
static void init_pairs(int k)
{
    int q = 0;
    for (int i = 0; i < k; i++)
        for (int j = i + 1; j < k; j++) { pair_idx[i][j] = q; pair_idx[j][i] = q; pair_i[q] = i; pair_j[q] = j; q++; }
}

static uint32_t permute_code(uint32_t code, const int *perm, int k)
{
    /* new graph: position i holds old vertex perm[i]; old pair {a, b} lands on
       the pair of the positions of a and b */
    int pos[KMAX];
    for (int i = 0; i < k; i++) pos[perm[i]] = i;
    uint32_t out = 0;
    while (code) {
        int q = __builtin_ctz(code);
        code &= code - 1;
        out |= 1u << pair_idx[pos[pair_i[q]]][pos[pair_j[q]]];
    }
    return out;
}

static int connected_code(uint32_t code, int k)
{
    unsigned seen = 1, frontier = 1;
    while (frontier) {
        unsigned nf = 0;
        for (int i = 0; i < k; i++) if (frontier >> i & 1)
            for (int j = 0; j < k; j++) if (j != i && (code >> pair_idx[i][j] & 1u) && !(seen >> j & 1)) { seen |= 1u << j; nf |= 1u << j; }
        frontier = nf;
    }
    return seen == (1u << k) - 1;
}

static int next_perm(int *a, int n)
{
    int i = n - 2;
    while (i >= 0 && a[i] >= a[i + 1]) i--;
    if (i < 0) return 0;
    int j = n - 1;
    while (a[j] <= a[i]) j--;
    int t = a[i]; a[i] = a[j]; a[j] = t;
    for (int l = i + 1, r = n - 1; l < r; l++, r--) { t = a[l]; a[l] = a[r]; a[r] = t; }
    return 1;
}

static uint32_t canonical_code(uint32_t code, int k)
{
    int p[KMAX];
    for (int i = 0; i < k; i++) p[i] = i;
    uint32_t best = 0xFFFFFFFFu;
    do {
        uint32_t c = permute_code(code, p, k);
        if (c < best) best = c;
    } while (next_perm(p, k));
    return best;
}

uint32_t orc_canonical_code(uint32_t code, int k) { init_pairs(k); return canonical_code(code, k); }

/* catalog: canonical codes of all connected graphs on k vertices, ascending */
static uint32_t *cat_codes[KMAX + 1];
static int cat_n[KMAX + 1];

static int build_catalog(int k)
{
    if (cat_codes[k]) return ORC_OK;
    init_pairs(k);
    int nb = k * (k - 1) / 2;
    uint64_t ncodes = 1ull << nb;
    uint8_t *seen = calloc((ncodes + 7) / 8, 1);
    if (!seen) return ORC_ENOMEM;
    int cap = 16, cnt = 0;
    uint32_t *codes = malloc(cap * sizeof(uint32_t));
    int p[KMAX];
    for (uint64_t c = 0; c < ncodes; c++) {
        if (seen[c >> 3] >> (c & 7) & 1) continue;
        if (!connected_code((uint32_t)c, k)) continue;
        /* the first unseen code of a connected orbit is its minimum */
        if (cnt == cap) { cap *= 2; codes = realloc(codes, cap * sizeof(uint32_t)); }
        codes[cnt++] = (uint32_t)c;
        for (int i = 0; i < k; i++) p[i] = i;
        do {
            uint32_t o = permute_code((uint32_t)c, p, k);
            seen[o >> 3] |= (uint8_t)(1u << (o & 7));
        } while (next_perm(p, k));
    }
    free(seen);
    cat_codes[k] = codes;
    cat_n[k] = cnt;
    return ORC_OK;
}

int orc_num_classes(int k)
{
    if (k < 1 || k > KMAX) return -1;
    if (build_catalog(k)) return -1;
    return cat_n[k];
}

int orc_catalog_codes(int k, uint32_t *out)
{
    if (build_catalog(k)) return ORC_ENOMEM;
    memcpy(out, cat_codes[k], cat_n[k] * sizeof(uint32_t));
    return ORC_OK;
}

static int class_of_code(int k, uint32_t canon)
{
    int lo = 0, hi = cat_n[k];
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (cat_codes[k][mid] == canon) return mid;
        if (cat_codes[k][mid] < canon) lo = mid + 1; else hi = mid;
    }
    return -1;
}

static int has_edge(const int64_t *row_ptr, const int32_t *col_idx, int64_t a, int64_t b)
{
    int64_t lo = row_ptr[a], hi = row_ptr[a + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (col_idx[mid] == b) return 1;
        if (col_idx[mid] < b) lo = mid + 1; else hi = mid;
    }
    return 0;
}

/* induced adjacency code of each sample, then its class id */
int orc_classify(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, int k,
                 const int32_t *verts, int64_t nsamp, uint32_t *out_code, int32_t *out_class)
{
    if (k < 2 || k > KMAX) return ORC_EINVAL;
    if (build_catalog(k)) return ORC_ENOMEM;
    init_pairs(k);
    for (int64_t s = 0; s < nsamp; s++) {
        const int32_t *vs = verts + s * k;
        uint32_t code = 0;
        for (int i = 0; i < k; i++)
            for (int j = i + 1; j < k; j++) {
                if (vs[i] < 0 || vs[i] >= n || vs[j] < 0 || vs[j] >= n) return ORC_EINVAL;
                if (has_edge(row_ptr, col_idx, vs[i], vs[j])) code |= 1u << pair_idx[i][j];
            }
        if (out_code) out_code[s] = code;
        out_class[s] = class_of_code(k, canonical_code(code, k));
    }
    return ORC_OK;
}

/* sigma_i: Kirchhoff's matrix-tree theorem, determinant by Bareiss elimination */
int64_t orc_spanning_trees(uint32_t code, int k)
{
    init_pairs(k);
    if (k == 1) return 1;
    int64_t L[KMAX][KMAX];
    memset(L, 0, sizeof L);
    for (int i = 0; i < k; i++)
        for (int j = 0; j < k; j++)
            if (i != j && (code >> pair_idx[i][j] & 1u)) { L[i][j] = -1; L[i][i]++; }
    /* minor: drop row and column 0 */
    int m = k - 1;
    int64_t A[KMAX][KMAX];
    for (int i = 0; i < m; i++) for (int j = 0; j < m; j++) A[i][j] = L[i + 1][j + 1];
    int64_t prev = 1;
    int sign = 1;
    for (int p = 0; p < m - 1; p++) {
        if (A[p][p] == 0) {
            int q = p + 1;
            while (q < m && A[q][p] == 0) q++;
            if (q == m) return 0;
            for (int j = 0; j < m; j++) { int64_t t = A[p][j]; A[p][j] = A[q][j]; A[q][j] = t; }
            sign = -sign;
        }
        for (int i = p + 1; i < m; i++)
            for (int j = p + 1; j < m; j++)
                A[i][j] = (A[i][j] * A[p][p] - A[i][p] * A[p][j]) / prev;
        prev = A[p][p];
    }
    return sign * A[m - 1][m - 1];
}

/* unrooted shape id of a tree on k labelled vertices given by a code */
static int tree_shape_id(uint32_t code, int k)
{
    tree_t t;
    memset(&t, 0, sizeof t);
    t.nn = k;
    for (int i = 0; i < k; i++)
        for (int j = i + 1; j < k; j++)
            if (code >> pair_idx[i][j] & 1u) { t.adj[i][t.deg[i]++] = j; t.adj[j][t.deg[j]++] = i; }
    int best = MAXSH;
    for (int x = 0; x < k; x++) {
        char s[SLEN];
        canon_at(&t, x, -1, s);
        int q = rank_of(k, s);
        if (q < best) best = q;
    }
    for (int j = 0; j < unr_n[k]; j++) if (unr_minrank[k][j] == best) return j;
    return -1;
}

/* sigma_ij: spanning trees of the graph with code `code` whose unrooted shape
   is j, by enumerating every (k-1)-subset of its edges */
int orc_spanning_trees_by_shape(uint32_t code, int k, int64_t *out /* unr_n[k] */)
{
    build_shapes();
    init_pairs(k);
    for (int j = 0; j < unr_n[k]; j++) out[j] = 0;
    int eu[32], ev[32], ne = 0;
    for (int i = 0; i < k; i++)
        for (int j = i + 1; j < k; j++)
            if (code >> pair_idx[i][j] & 1u) { eu[ne] = i; ev[ne] = j; ne++; }
    if (k == 1) { out[0] = 1; return ORC_OK; }
    int idx[KMAX];
    int r = k - 1;
    if (ne < r) return ORC_OK;
    for (int i = 0; i < r; i++) idx[i] = i;
    for (;;) {
        /* is this subset a spanning tree? union-find over its r edges */
        int par[KMAX];
        for (int i = 0; i < k; i++) par[i] = i;
        int ok = 1;
        uint32_t tc = 0;
        for (int i = 0; i < r && ok; i++) {
            int a = eu[idx[i]], b = ev[idx[i]];
            while (par[a] != a) a = par[a];
            while (par[b] != b) b = par[b];
            if (a == b) ok = 0; else par[a] = b;
            tc |= 1u << pair_idx[eu[idx[i]]][ev[idx[i]]];
        }
        if (ok) out[tree_shape_id(tc, k)]++;
        int i = r - 1;
        while (i >= 0 && idx[i] == ne - r + i) i--;
        if (i < 0) break;
        idx[i]++;
        for (int j = i + 1; j < r; j++) idx[j] = idx[j - 1] + 1;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* AGS (Sec. 4.1): rounds of `round_size` samples of one treelet shape.       */
/* Start with the most frequent shape (largest t_j, ties to the smaller id).   */
/* After each round: n_j += round size, c_i += hits. The algorithm's switch   */
/* test looks at the class just sampled: if its count has reached cbar, the   */
/* class joins the covered set (if it was not there) and the next shape is    */
/* chosen again, whether or not the cover is new. With rounds, that test is   */
/* made for every class the round hit; if any of them has c_i >= cbar, switch */
/* to                                                                          */
/*   j* = argmin_{j : t_j > 0} (1/t_j) sum_{i covered} sigma_ij c_i / w_i,     */
/* with w_i = sum_j n_j sigma_ij / t_j. Scores within a relative 2^-40 of the  */
/* best so far count as ties, and ties go to the smaller j (exactly equal     */
/* rationals must not be split by FP64 rounding). Stop when all classes are   */
/* covered or `budget` samples were drawn. Round r draws sample indices       */
/* [drawn, drawn + round_size) of (seed, stream); round_size = 1 is the       */
/* algorithm sample by sample.                                                 */
/* Outputs per class: hits c_i and w_i; the estimate of the colourful count   */
/* is c_i / w_i.                                                              */
/* ------------------------------------------------------------------------- */
int orc_ags(const orc_table *T, int64_t cbar, int64_t round_size, int64_t budget,
            uint64_t seed, uint64_t stream,
            int64_t *out_hits, double *out_w, int64_t *out_nj, int32_t *out_rounds_shape, int64_t *out_nrounds)
{
    if (T->rooting == ORC_ROOT_BALANCED) { set_err("AGS needs zero-rooting or all rootings"); return ORC_EINVAL; }
    const int k = T->k;
    int st = build_catalog(k);
    if (st) return st;
    build_shapes();
    const int s = cat_n[k], ns = unr_n[k];
    /* sigma_ij rows are computed when a class is first hit: only hit classes
       enter w_i, the covered sums and the outputs */
    int64_t *sig = calloc((size_t)s * ns, sizeof(int64_t));
    char *sig_ok = calloc(s, 1);
    int64_t *c = calloc(s, sizeof(int64_t));
    double *w = calloc(s, sizeof(double));
    int64_t *nj = calloc(ns, sizeof(int64_t));
    char *cov = calloc(s, 1);
    char *hit = calloc(s, 1);
    int32_t *verts = malloc(round_size * k * sizeof(int32_t));
    int8_t *par = malloc(round_size * k);
    int32_t *cls = malloc(round_size * sizeof(int32_t));
    double tjd[64];
    for (int j = 0; j < ns; j++) tjd[j] = (double)T->tj[j];

    int j = -1;
    int64_t drawn = 0, nr = 0, ncov = 0;
    for (int q = 0; q < ns; q++) if (T->tj[q] > 0 && (j < 0 || T->tj[q] > T->tj[j])) j = q;
    if (j < 0) { st = ORC_EEMPTY; set_err("no colourful k-treelet"); goto done; }
    while (ncov < s && drawn + round_size <= budget) {
        st = orc_sample(T, j, round_size, seed, stream, (uint64_t)drawn, verts, par);
        if (st) goto done;
        st = orc_classify(T->n, T->row_ptr, T->col_idx, k, verts, round_size, NULL, cls);
        if (st) goto done;
        if (out_rounds_shape) out_rounds_shape[nr] = j;
        nr++;
        drawn += round_size;
        nj[j] += round_size;
        for (int64_t q = 0; q < round_size; q++) {
            int i = cls[q];
            if (i < 0) { st = ORC_EINVAL; set_err("internal: unclassified sample"); goto done; }
            c[i]++;
            hit[i] = 1;
            if (!sig_ok[i]) { orc_spanning_trees_by_shape(cat_codes[k][i], k, sig + (size_t)i * ns); sig_ok[i] = 1; }
        }
        int reselect = 0;
        for (int i = 0; i < s; i++) {
            if (hit[i] && c[i] >= cbar) {
                reselect = 1;
                if (!cov[i]) { cov[i] = 1; ncov++; }
            }
            hit[i] = 0;
        }
        if (reselect && ncov < s) {
            for (int i = 0; i < s; i++) {
                if (!cov[i]) continue;
                double acc = 0.0;
                for (int q = 0; q < ns; q++)
                    if (tjd[q] > 0) acc += (double)nj[q] * (double)sig[(size_t)i * ns + q] / tjd[q];
                w[i] = acc;
            }
            int best = -1;
            double bv = 0.0;
            for (int q = 0; q < ns; q++) {
                if (!(tjd[q] > 0)) continue;
                double acc = 0.0;
                for (int i = 0; i < s; i++)
                    if (cov[i]) acc += (double)sig[(size_t)i * ns + q] * (double)c[i] / w[i];
                acc /= tjd[q];
                if (best < 0 || acc < bv * (1.0 - 0x1p-40)) { best = q; bv = acc; }
            }
            j = best;
        }
    }
    for (int i = 0; i < s; i++) {
        double acc = 0.0;
        if (sig_ok[i])
            for (int q = 0; q < ns; q++)
                if (tjd[q] > 0) acc += (double)nj[q] * (double)sig[(size_t)i * ns + q] / tjd[q];
        out_hits[i] = c[i];
        out_w[i] = acc;
    }
    for (int q = 0; q < ns; q++) out_nj[q] = nj[q];
    *out_nrounds = nr;
    st = ORC_OK;
done:
    free(sig); free(sig_ok); free(c); free(w); free(nj); free(cov); free(hit); free(verts); free(par); free(cls);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Estimators (Sec. 2.2). A uniform colourful k-treelet copy spans graphlet  */
/* H_i with probability c_i sigma_i / t, where c_i counts the colourful       */
/* copies of H_i and sigma_i its spanning trees; so with hits_i of n samples */
/* in class i,  c_i ~= t (hits_i / n) / sigma_i.  AGS (Sec. 4.1) gives        */
/* c_i ~= hits_i / w_i instead (w given; 0 where w_i = 0). A colourful        */
/* k-subset has probability p_k, so the copies in G are g_i ~= c_i / p_k     */
/* (p_k <= 0 here: the uniform colouring's k!/k^k).                          */
/* ------------------------------------------------------------------------- */
int orc_estimate(const orc_table *T, const int64_t *hits, const double *w, int64_t n, double pk,
                 double *out_c, double *out_g)
{
    const int k = T->k;
    int st = build_catalog(k);
    if (st) return st;
    if (!hits || (!w && n <= 0)) { set_err("bad estimator input"); return ORC_EINVAL; }
    if (pk <= 0) {
        pk = 1.0;
        for (int i = 1; i <= k; i++) pk *= (double)i / (double)k;
    }
    const double t = (double)T->t;
    for (int i = 0; i < cat_n[k]; i++) {
        double c;
        if (w) c = w[i] > 0 ? (double)hits[i] / w[i] : 0.0;
        else c = t * ((double)hits[i] / (double)n) / (double)orc_spanning_trees(cat_codes[k][i], k);
        if (out_c) out_c[i] = c;
        if (out_g) out_g[i] = c / pk;
    }
    return ORC_OK;
}
