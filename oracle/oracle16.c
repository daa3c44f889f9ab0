/*
 * oracle16.c -- TEST INFRASTRUCTURE ONLY. The build-up dynamic program for
 * k up to 16 (the generality of Sec. 3.2, "Treelet representation" and
 * "Count tables"), as plain single-threaded C with sparse records.
 *
 * A rooted treelet on h nodes is its DFS bitstring of 2(h-1) bits (Sec. 3.2:
 * '1' for an edge taken away from the root, '0' for the way back, children in
 * descending lexicographic order of their words "1 s 0"), held in a uint32
 * with the first edge at bit 2(h-1)-1. A coloured treelet (T, C) is the 46-bit
 * key s_T << 16 | C, C the colour set as a k-bit mask (h = |C|). A vertex's
 * level-h record is the list of its non-zero counts sorted by key (Sec. 3.2,
 * "Count tables"); counts are unsigned 256-bit integers (four 64-bit words),
 * every add and multiply checked.
 *
 * Level h at v (Eq. (1)): for every pair of a record entry (T', C') of v of
 * some size h' and an entry (T'', C'') of v's neighbour sum S_{h-h'}(v) =
 * sum over u ~ v of u's level-(h-h') records restricted to colour sets without
 * c_v, with C' and C'' disjoint and the word of T'' not smaller than any root
 * child word of T' (so that T'' becomes a largest root child: each T arises
 * from exactly one such pair), add the product to (T' with T'' attached to its
 * root, C' | C''); then divide each sum by beta_T, the number of root children
 * of T equal to T'' (reading 2 of the oracle). Level k is kept at colour-0
 * vertices (zero-rooting, Sec. 3.4) or at every vertex; t is their sum (divided
 * by k for all rootings).
 *
 * Pinned (tests/test_oracle16.py) by brute-force subtree enumeration at
 * k = 9 and 10 (and on a path at k = 16), by the star's closed form (products
 * of colour class sizes) at k = 12 and 16, and by equality with the k <= 8
 * oracle's tables for k = 3..8.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* Unsigned 256-bit counts: four 64-bit words, least significant first. */
typedef struct { uint64_t w[4]; } u256;

static u256 u256_of(uint64_t x)
{
    u256 r = {{x, 0, 0, 0}};
    return r;
}
static int u256_is_zero(u256 a) { return !(a.w[0] | a.w[1] | a.w[2] | a.w[3]); }

/* *r = a + b; nonzero when the sum needs more than 256 bits */
static int u256_add(u256 *r, u256 a, u256 b)
{
    u128 c = 0;
    for (int i = 0; i < 4; i++) {
        c += (u128)a.w[i] + b.w[i];
        r->w[i] = (uint64_t)c;
        c >>= 64;
    }
    return c != 0;
}

/* *r = a * b, schoolbook on 64-bit words; nonzero when the product needs more
 * than 256 bits */
static int u256_mul(u256 *r, u256 a, u256 b)
{
    uint64_t p[8] = {0};
    for (int i = 0; i < 4; i++) {
        u128 c = 0;
        for (int j = 0; j < 4; j++) {
            c += (u128)a.w[i] * b.w[j] + p[i + j];
            p[i + j] = (uint64_t)c;
            c >>= 64;
        }
        p[i + 4] = (uint64_t)c;
    }
    for (int i = 0; i < 4; i++) r->w[i] = p[i];
    return (p[4] | p[5] | p[6] | p[7]) != 0;
}

/* *q = a / d (d > 0); returns the remainder */
static uint64_t u256_divmod(u256 *q, u256 a, uint64_t d)
{
    u128 r = 0;
    for (int i = 3; i >= 0; i--) {
        r = (r << 64) | a.w[i];
        q->w[i] = (uint64_t)(r / d);
        r %= d;
    }
    return (uint64_t)r;
}

/* The arithmetic above on caller-given words (a test hook for the pins):
 * sum = a + b, prod = a * b, quot = a / d, *rem = a mod d; flags bit 0: the sum
 * overflowed, bit 1: the product overflowed. */
void orc16_u256_ops(const uint64_t a[4], const uint64_t b[4], uint64_t d, uint64_t sum[4], uint64_t prod[4],
                    uint64_t quot[4], uint64_t *rem, int *flags)
{
    u256 x, y, r;
    for (int i = 0; i < 4; i++) { x.w[i] = a[i]; y.w[i] = b[i]; }
    *flags = 0;
    if (u256_add(&r, x, y)) *flags |= 1;
    for (int i = 0; i < 4; i++) sum[i] = r.w[i];
    if (u256_mul(&r, x, y)) *flags |= 2;
    for (int i = 0; i < 4; i++) prod[i] = r.w[i];
    *rem = u256_divmod(&r, x, d);
    for (int i = 0; i < 4; i++) quot[i] = r.w[i];
}

#define K16 16
#define O16_OK 0
#define O16_EINVAL -1
#define O16_ENOMEM -2
#define O16_EOVERFLOW -3

static char o16_err[256];
const char *orc16_last_error(void) { return o16_err; }

typedef struct { uint64_t key; u256 cnt; } ent;
typedef struct { ent *e; int64_t len, cap; } rec;

static int rec_push(rec *r, uint64_t key, u256 cnt)
{
    if (r->len == r->cap) {
        int64_t nc = r->cap ? 2 * r->cap : 8;
        ent *ne = realloc(r->e, (size_t)nc * sizeof(ent));
        if (!ne) return O16_ENOMEM;
        r->e = ne;
        r->cap = nc;
    }
    r->e[r->len].key = key;
    r->e[r->len].cnt = cnt;
    r->len++;
    return O16_OK;
}

static int cmp_ent(const void *a, const void *b)
{
    uint64_t x = ((const ent *)a)->key, y = ((const ent *)b)->key;
    return x < y ? -1 : x > y;
}

/* sorts by key and adds the counts of equal keys; zeros dropped */
static int rec_normalise(rec *r)
{
    if (r->len == 0) return O16_OK;
    qsort(r->e, (size_t)r->len, sizeof(ent), cmp_ent);
    int64_t w = 0;
    for (int64_t i = 0; i < r->len; i++) {
        if (w > 0 && r->e[w - 1].key == r->e[i].key) {
            if (u256_add(&r->e[w - 1].cnt, r->e[w - 1].cnt, r->e[i].cnt)) return O16_EOVERFLOW;
        } else {
            r->e[w++] = r->e[i];
        }
    }
    int64_t z = 0;
    for (int64_t i = 0; i < w; i++)
        if (!u256_is_zero(r->e[i].cnt)) r->e[z++] = r->e[i];
    r->len = z;
    return O16_OK;
}

/* ------------------------------------------------------------------------- */
/* Bitstrings: a string of len bits, first bit at position len-1.              */
/* ------------------------------------------------------------------------- */
static int bit_at(uint32_t s, int len, int i) { return (int)((s >> (len - 1 - i)) & 1u); }

/* lexicographic comparison ('0' < '1'; a proper prefix is smaller) */
static int cmp_str(uint32_t a, int la, uint32_t b, int lb)
{
    int m = la < lb ? la : lb;
    for (int i = 0; i < m; i++) {
        int x = bit_at(a, la, i), y = bit_at(b, lb, i);
        if (x != y) return x < y ? -1 : 1;
    }
    return la < lb ? -1 : la > lb;
}

/* the root's child words "1 s 0" of a rooted treelet, in their stored order */
static int child_words(uint32_t s, int len, uint32_t *w, int *wl)
{
    int nw = 0, depth = 0, start = 0;
    for (int i = 0; i < len; i++) {
        depth += bit_at(s, len, i) ? 1 : -1;
        if (depth == 0) {
            int l = i - start + 1;
            w[nw] = (s >> (len - 1 - i)) & (l == 32 ? 0xffffffffu : ((1u << l) - 1u));
            wl[nw] = l;
            nw++;
            start = i + 1;
        }
    }
    return nw;
}

/* T' with T'' attached as one more root child: returns the merged string in
 * *out (length lp + lpp + 2) and beta_T, or 0 when T'' is not a largest child */
static int merge_shapes(uint32_t sp, int lp, uint32_t spp, int lpp, uint32_t *out)
{
    uint32_t w[K16], word = (1u << (lpp + 1)) | (spp << 1);
    int wl[K16], nw = child_words(sp, lp, w, wl), lw = lpp + 2;
    for (int i = 0; i < nw; i++)
        if (cmp_str(word, lw, w[i], wl[i]) < 0) return 0;
    /* the new word goes first; the others keep their (descending) order */
    uint32_t s = word;
    int beta = 1;
    for (int i = 0; i < nw; i++) {
        s = (s << wl[i]) | w[i];
        if (wl[i] == lw && w[i] == word) beta++;
    }
    *out = s;
    return beta;
}

static uint64_t make_key(uint32_t s, uint32_t C) { return ((uint64_t)s << 16) | C; }
static uint32_t key_shape(uint64_t key) { return (uint32_t)(key >> 16); }
static uint32_t key_colours(uint64_t key) { return (uint32_t)(key & 0xffffu); }

/* ------------------------------------------------------------------------- */
/* The table                                                                 */
/* ------------------------------------------------------------------------- */
typedef struct orc16_table {
    int k, rooting;
    int64_t n;
    rec *X[K16 + 1];   /* [n] per level */
    u256 t;
} orc16_table;

void orc16_table_free(orc16_table *T)
{
    if (!T) return;
    for (int h = 1; h <= K16; h++) {
        if (!T->X[h]) continue;
        for (int64_t v = 0; v < T->n; v++) free(T->X[h][v].e);
        free(T->X[h]);
    }
    free(T);
}

int orc16_build(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const uint8_t *colors, int k,
                int rooting, orc16_table **out)
{
    *out = NULL;
    if (k < 2 || k > K16 || n < 0 || (rooting != 0 && rooting != 1)) {
        snprintf(o16_err, sizeof o16_err, "bad arguments (k = %d)", k);
        return O16_EINVAL;
    }
    for (int64_t v = 0; v < n; v++)
        if (colors[v] >= k) { snprintf(o16_err, sizeof o16_err, "colour >= k"); return O16_EINVAL; }
    orc16_table *T = calloc(1, sizeof *T);
    if (!T) return O16_ENOMEM;
    T->k = k; T->rooting = rooting; T->n = n;
    rec *S[K16 + 1] = {0};
    int st = O16_OK;
    for (int h = 1; h <= k && !st; h++) {
        T->X[h] = calloc((size_t)(n ? n : 1), sizeof(rec));
        if (!T->X[h]) { st = O16_ENOMEM; break; }
    }
    /* level 1: the single node coloured c_v, once */
    for (int64_t v = 0; v < n && !st; v++) st = rec_push(&T->X[1][v], make_key(0, 1u << colors[v]), u256_of(1));
    for (int h = 2; h <= k && !st; h++) {
        /* neighbour sums of level h-1 */
        const int hs = h - 1;
        S[hs] = calloc((size_t)(n ? n : 1), sizeof(rec));
        if (!S[hs]) { st = O16_ENOMEM; break; }
        for (int64_t v = 0; v < n && !st; v++) {
            const uint32_t cvb = 1u << colors[v];
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1] && !st; e++) {
                const rec *ru = &T->X[hs][col_idx[e]];
                for (int64_t i = 0; i < ru->len && !st; i++)
                    if (!(key_colours(ru->e[i].key) & cvb)) st = rec_push(&S[hs][v], ru->e[i].key, ru->e[i].cnt);
            }
            if (!st) st = rec_normalise(&S[hs][v]);
        }
        /* Eq. (1) */
        for (int64_t v = 0; v < n && !st; v++) {
            if (h == k && rooting == 0 && colors[v] != 0) continue;
            rec acc = {0}, beta = {0};
            for (int hp = 1; hp < h && !st; hp++) {
                const rec *x = &T->X[hp][v], *s = &S[h - hp][v];
                for (int64_t i = 0; i < x->len && !st; i++)
                    for (int64_t j = 0; j < s->len && !st; j++) {
                        const uint32_t Cp = key_colours(x->e[i].key), Cpp = key_colours(s->e[j].key);
                        if (Cp & Cpp) continue;
                        uint32_t sT;
                        const int b = merge_shapes(key_shape(x->e[i].key), 2 * (hp - 1), key_shape(s->e[j].key),
                                                   2 * (h - hp - 1), &sT);
                        if (!b) continue;
                        u256 p;
                        if (u256_mul(&p, x->e[i].cnt, s->e[j].cnt)) st = O16_EOVERFLOW;
                        else st = rec_push(&acc, make_key(sT, Cp | Cpp), p);
                        if (!st) st = rec_push(&beta, make_key(sT, Cp | Cpp), u256_of((uint64_t)b));
                    }
            }
            if (!st) st = rec_normalise(&acc);
            if (!st) {
                /* beta depends on T alone: look it up in the (sorted) list of pairs seen */
                if (beta.len) qsort(beta.e, (size_t)beta.len, sizeof(ent), cmp_ent);
                int64_t q = 0;
                for (int64_t i = 0; i < acc.len && !st; i++) {
                    while (beta.e[q].key != acc.e[i].key) q++;
                    const uint64_t b = beta.e[q].cnt.w[0];
                    if (u256_divmod(&acc.e[i].cnt, acc.e[i].cnt, b)) {
                        snprintf(o16_err, sizeof o16_err, "beta does not divide a sum");
                        st = O16_EINVAL;
                    }
                }
            }
            free(beta.e);
            if (st) { free(acc.e); break; }
            T->X[h][v] = acc;
        }
        if (st == O16_EOVERFLOW) snprintf(o16_err, sizeof o16_err, "a count needs more than 256 bits");
    }
    for (int h = 1; h <= K16; h++) {
        if (!S[h]) continue;
        for (int64_t v = 0; v < n; v++) free(S[h][v].e);
        free(S[h]);
    }
    if (!st) {
        u256 t = u256_of(0);
        for (int64_t v = 0; v < n && !st; v++)
            for (int64_t i = 0; i < T->X[k][v].len && !st; i++)
                if (u256_add(&t, t, T->X[k][v].e[i].cnt)) st = O16_EOVERFLOW;
        if (!st && rooting == 1 && u256_divmod(&t, t, (uint64_t)k)) {
            snprintf(o16_err, sizeof o16_err, "k does not divide the level-k total");
            st = O16_EINVAL;
        }
        T->t = t;
    }
    if (st) { orc16_table_free(T); return st; }
    *out = T;
    return O16_OK;
}

int64_t orc16_level_nnz(const orc16_table *T, int h)
{
    if (h < 1 || h > T->k) return -1;
    int64_t s = 0;
    for (int64_t v = 0; v < T->n; v++) s += T->X[h][v].len;
    return s;
}

/* level h in vertex order: off[n+1], key[nnz] (s_T << 16 | C), counts as four
 * words each, least significant first (words[4 * i .. 4 * i + 3]) */
int orc16_export_level(const orc16_table *T, int h, int64_t *off, uint64_t *key, uint64_t *words)
{
    if (h < 1 || h > T->k) return O16_EINVAL;
    int64_t at = 0;
    for (int64_t v = 0; v < T->n; v++) {
        off[v] = at;
        const rec *r = &T->X[h][v];
        for (int64_t i = 0; i < r->len; i++, at++) {
            key[at] = r->e[i].key;
            for (int q = 0; q < 4; q++) words[4 * at + q] = r->e[i].cnt.w[q];
        }
    }
    off[T->n] = at;
    return O16_OK;
}

/* t as four words, least significant first */
void orc16_total(const orc16_table *T, uint64_t t[4])
{
    for (int q = 0; q < 4; q++) t[q] = T->t.w[q];
}
