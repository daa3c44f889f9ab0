// Host-side treelet algebra of libscc: rooted shapes, canonical decompositions,
// unrooted shape ids and the per-k lookup tables used by the kernels.
//
// A rooted tree is its DFS bitstring (Sec. 3.2): '1' for an edge taken away
// from the root, '0' for the way back, children visited in descending
// lexicographic order of their words "1 s 0". Shapes of one size are ranked
// by ascending bitstring. The canonical decomposition takes the first child
// subtree as T'' and the rest as T' (the merge is 1, s_T'', 0, s_T'); beta_T
// is the number of children equal to that first child.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>

#include "scc_common.hpp"

namespace {

struct Word {          // a child word "1 s 0" or a shape string, MSB first
    uint32_t bits;
    int len;
};

// lexicographic comparison of two bitstrings of possibly different length;
// child words are primitive balanced strings, so neither is a prefix of the other
bool word_less(const Word &a, const Word &b)
{
    uint64_t x = a.len ? (uint64_t)a.bits << (64 - a.len) : 0;
    uint64_t y = b.len ? (uint64_t)b.bits << (64 - b.len) : 0;
    if (x != y) return x < y;
    return a.len < b.len;
}

Word concat(const Word &a, const Word &b)
{
    return Word{(a.bits << b.len) | b.bits, a.len + b.len};
}

HostShapes g_shapes;
int g_unr_n[SCC_KMAX + 1];
int g_unr_of[SCC_KMAX + 1][SCC_MAXSH];
int g_unr_min[SCC_KMAX + 1][SCC_MAXSH];
std::once_flag g_once;

int rank_of(int h, uint32_t bits)
{
    const uint32_t *b = g_shapes.bits[h];
    int n = g_shapes.r[h];
    const uint32_t *p = std::lower_bound(b, b + n, bits);
    return (p != b + n && *p == bits) ? (int)(p - b) : -1;
}

// Canonical string of the tree hanging at v (entered from p) over adjacency masks.
Word canon(const uint32_t *adj, int v, int p)
{
    Word kids[SCC_KMAX + 8];
    int nk = 0;
    for (uint32_t m = adj[v]; m; m &= m - 1) {
        int w = __builtin_ctz(m);
        if (w == p) continue;
        Word in = canon(adj, w, v);
        kids[nk++] = Word{(1u << (in.len + 1)) | (in.bits << 1), in.len + 2};
    }
    std::sort(kids, kids + nk, [](const Word &a, const Word &b) { return word_less(b, a); });
    Word s{0, 0};
    for (int i = 0; i < nk; i++) s = concat(s, kids[i]);
    return s;
}

// adjacency masks of the rooted tree with the given string (node 0 = root)
int parse(uint32_t bits, int len, uint32_t *adj)
{
    int stack[16], sp = 0, nn = 1;
    adj[0] = 0;
    stack[sp++] = 0;
    for (int i = len - 1; i >= 0; i--) {
        if (bits >> i & 1u) {
            int x = nn++;
            adj[x] = 0;
            int p = stack[sp - 1];
            adj[p] |= 1u << x;
            adj[x] |= 1u << p;
            stack[sp++] = x;
        } else {
            sp--;
        }
    }
    return nn;
}

void init_shapes()
{
    // words[s]: all child words of subtrees with s nodes, i.e. "1 s_T 0" for |T| = s
    std::vector<Word> words[SCC_KMAX + 1];
    g_shapes.r[1] = 1;
    g_shapes.bits[1][0] = 0;
    words[1].push_back(Word{0b10, 2});
    for (int h = 2; h <= SCC_KMAX; h++) {
        // children multisets with sizes summing to h-1, in non-increasing word order
        std::vector<uint32_t> found;
        std::vector<Word> cur;
        std::function<void(int, bool, Word)> rec = [&](int remaining, bool bounded, Word maxw) {
            if (remaining == 0) {
                Word s{0, 0};
                for (const Word &w : cur) s = concat(s, w);
                found.push_back(s.bits);
                return;
            }
            for (int s = 1; s <= remaining; s++)
                for (const Word &w : words[s]) {
                    if (bounded && word_less(maxw, w)) continue;
                    cur.push_back(w);
                    rec(remaining - s, true, w);
                    cur.pop_back();
                }
        };
        rec(h - 1, false, Word{0, 0});
        std::sort(found.begin(), found.end());
        found.erase(std::unique(found.begin(), found.end()), found.end());
        g_shapes.r[h] = (int)found.size();
        for (size_t i = 0; i < found.size(); i++) {
            g_shapes.bits[h][i] = found[i];
            words[h].push_back(Word{(1u << (2 * h - 1)) | (found[i] << 1), 2 * h});
        }
    }
    // unrooted classes: minimum rooted rank over all rootings, numbered ascending
    for (int h = 1; h <= SCC_KMAX; h++) {
        int minr[SCC_MAXSH];
        for (int q = 0; q < g_shapes.r[h]; q++) {
            uint32_t adj[16];
            int nn = parse(g_shapes.bits[h][q], 2 * (h - 1), adj);
            int best = SCC_MAXSH;
            for (int x = 0; x < nn; x++) best = std::min(best, rank_of(h, canon(adj, x, -1).bits));
            minr[q] = best;
        }
        std::vector<int> mins(minr, minr + g_shapes.r[h]);
        std::sort(mins.begin(), mins.end());
        mins.erase(std::unique(mins.begin(), mins.end()), mins.end());
        g_unr_n[h] = (int)mins.size();
        for (size_t j = 0; j < mins.size(); j++) g_unr_min[h][j] = mins[j];
        for (int q = 0; q < g_shapes.r[h]; q++)
            g_unr_of[h][q] = (int)(std::lower_bound(mins.begin(), mins.end(), minr[q]) - mins.begin());
    }
}

int binom(int n, int r)
{
    if (r < 0 || r > n) return 0;
    long v = 1;
    for (int i = 1; i <= r; i++) v = v * (n - r + i) / i;
    return (int)v;
}

}  // namespace

const HostShapes &host_shapes()
{
    std::call_once(g_once, init_shapes);
    return g_shapes;
}

int unrooted_count(int k)
{
    host_shapes();
    return g_unr_n[k];
}

int tree_unrooted_id(int k, const uint32_t *adjmask)
{
    host_shapes();
    int best = SCC_MAXSH;
    for (int x = 0; x < k; x++) best = std::min(best, rank_of(k, canon(adjmask, x, -1).bits));
    for (int j = 0; j < g_unr_n[k]; j++)
        if (g_unr_min[k][j] == best) return j;
    return -1;
}

void build_lut(int k, DevLut *L)
{
    const HostShapes &S = host_shapes();
    memset(L, 0, sizeof *L);
    L->k = k;
    L->off[1] = 0;
    for (int h = 1; h <= k; h++) {
        L->r[h] = S.r[h];
        L->bk[h] = binom(k, h);
        L->bk1[h] = binom(k - 1, h);
        L->W[h] = S.r[h] * binom(k - 1, h - 1);
        L->WS[h] = S.r[h] * binom(k - 1, h);
        L->off[h + 1] = L->off[h] + S.r[h] * binom(k, h);
    }
    L->nkeys = L->off[k + 1];
    L->xoff[1] = 0;
    L->soff[1] = 0;
    for (int h = 1; h <= k; h++) {
        L->xoff[h + 1] = L->xoff[h] + L->W[h];
        L->soff[h + 1] = L->soff[h] + L->WS[h];
    }
    for (int h = 2; h <= k; h++)
        for (int q = 0; q < S.r[h]; q++) {
            uint32_t s = S.bits[h][q];
            int len = 2 * (h - 1);
            // first child word: scan to the first return to depth 0
            int depth = 0, wl = 0;
            for (int i = len - 1; i >= 0; i--) {
                depth += (s >> i & 1u) ? 1 : -1;
                if (depth == 0) { wl = len - i; break; }
            }
            uint32_t first = s >> (len - wl);
            uint32_t rest = s & ((wl == len) ? 0u : ((1u << (len - wl)) - 1u));
            int hpp = wl / 2, hp = h - hpp;
            uint32_t inner = (first >> 1) & ((1u << (wl - 2)) - 1u);
            // beta: children equal to the first word
            int beta = 0;
            depth = 0;
            int start = len;
            for (int i = len - 1; i >= 0; i--) {
                depth += (s >> i & 1u) ? 1 : -1;
                if (depth == 0) {
                    int l = start - i;
                    uint32_t w = (s >> i) & ((1u << l) - 1u);
                    if (l == wl && w == first) beta++;
                    start = i;
                }
            }
            L->dec_hp[h][q] = (uint8_t)hp;
            L->dec_a[h][q] = (uint8_t)rank_of(hp, rest);
            L->dec_b[h][q] = (uint8_t)rank_of(hpp, inner);
            L->dec_beta[h][q] = (uint8_t)beta;
        }
    L->num_unr = g_unr_n[k];
    for (int q = 0; q < S.r[k]; q++) L->unr_of[q] = (uint8_t)g_unr_of[k][q];
    // designated (balanced) rootings and their orbits
    uint32_t star = 0;
    for (int i = 0; i < k - 1; i++) star = (star << 2) | 2u;
    L->star_unr = k >= 2 ? g_unr_of[k][rank_of(k, star)] : 0;
    for (int j = 0; j < 32; j++) { L->bal_rank[j] = -1; L->bal_orbit[j] = 0; }
    for (int q = 0; k >= 4 && q < S.r[k]; q++) {
        const int hpp = k - L->dec_hp[k][q];
        if (hpp < 2 || hpp > k - 2) continue;
        int8_t &b = L->bal_rank[g_unr_of[k][q]];
        if (b < 0 || q < b) b = (int8_t)q;
    }
    for (int j = 0; j < L->num_unr; j++) {
        if (L->bal_rank[j] < 0) continue;
        L->designated[L->bal_rank[j]] = 1;
        uint32_t adj[16];
        const int nn = parse(S.bits[k][L->bal_rank[j]], 2 * (k - 1), adj);
        for (int x = 0; x < nn; x++) L->bal_orbit[j] += rank_of(k, canon(adj, x, -1).bits) == L->bal_rank[j];
    }
    int cnt[SCC_KMAX + 1] = {0};
    for (uint32_t m = 0; m < (1u << (k - 1)); m++) {
        int p = __builtin_popcount(m);
        L->colex_s[m] = (uint8_t)cnt[p];
        L->mask_s[p][cnt[p]++] = (uint8_t)m;
    }
    int cntk[SCC_KMAX + 2] = {0};
    for (uint32_t m = 0; m < (1u << k); m++) {
        int p = __builtin_popcount(m);
        L->colex_k[m] = (uint8_t)cntk[p];
        L->mask_k[p][cntk[p]++] = (uint8_t)m;
    }
    int nt = 0;
    for (int h = 2; h <= k; h++)
        for (int hp = 1; hp < h; hp++) {
            L->term_base[h][hp] = (uint16_t)nt;
            int nd = binom(k - 1, h - 1);
            for (int dc = 0; dc < nd; dc++) {
                uint32_t D = L->mask_s[h - 1][dc];
                for (uint32_t sub = 0; sub < (1u << (k - 1)); sub++) {
                    if ((sub & ~D) || __builtin_popcount(sub) != hp - 1) continue;
                    L->term_x[nt] = L->colex_s[sub];
                    L->term_s[nt] = L->colex_s[D ^ sub];
                    nt++;
                }
            }
        }
    for (int i = 0; i < nt; i++) L->term_xs[i] = (uint16_t)(L->term_x[i] | (L->term_s[i] << 8));
    // per-output descriptors and keys of every level
    uint32_t no = 0;
    for (int h = 2; h <= k; h++) {
        L->out_off[h] = no;
        const int nD = L->bk1[h - 1];
        for (int o = 0; o < L->W[h]; o++, no++) {
            const int t = o / nD, dc = o - t * nD;
            const int hp = L->dec_hp[h][t], hpp = h - hp;
            const uint64_t xb = (uint64_t)(L->xoff[hp] + L->dec_a[h][t] * L->bk1[hp - 1]);
            const uint64_t sb = (uint64_t)(L->soff[hpp] + L->dec_b[h][t] * L->bk1[hpp]);
            const uint64_t nsplit = (uint64_t)binom(h - 1, hp - 1);
            const uint64_t tb = L->term_base[h][hp] + (uint64_t)dc * nsplit;
            const uint64_t desig = (h == k && L->designated[t]) ? 1u : 0u;
            L->out[no] = xb | (sb << 16) | (tb << 32) | (nsplit << 48) | ((uint64_t)L->dec_beta[h][t] << 56) | (desig << 63);
            const uint32_t D = L->mask_s[h - 1][dc];
            for (int c = 0; c < k; c++) {
                const uint32_t C = expand_in(D, c) | (1u << c);
                L->out_key[c][no] = (uint16_t)(L->off[h] + t * L->bk[h] + L->colex_k[C]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local char t_err[512];

scc_status set_error(scc_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_err, sizeof t_err, fmt, ap);
    va_end(ap);
    return st;
}

extern "C" const char *scc_last_error(void) { return t_err; }
extern "C" const char *scc_version(void) { return "scc-mi355x 0.1 (gfx950)"; }
extern "C" int scc_num_unrooted(int k) { return (k >= 1 && k <= SCC_KMAX) ? unrooted_count(k) : -1; }

extern "C" int scc_balanced_rooting(int k, int j, int *orbit)
{
    if (orbit) *orbit = 0;
    if (k < 1 || k > SCC_KMAX || j < 0 || j >= unrooted_count(k)) return -1;
    std::unique_ptr<DevLut> L(new DevLut);   // ~50 KB: not on the caller's stack
    build_lut(k, L.get());
    if (orbit) *orbit = L->bal_orbit[j];
    return L->bal_rank[j];
}

extern "C" int scc_star_shape(int k)
{
    if (k < 2 || k > SCC_KMAX) return -1;
    std::unique_ptr<DevLut> L(new DevLut);
    build_lut(k, L.get());
    return L->star_unr;
}

void *DevMem::get(size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (alloc && alloc->alloc) return alloc->alloc(bytes, (void *)stream, alloc->ctx);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void DevMem::put(void *p)
{
    if (!p) return;
    if (alloc && alloc->free) alloc->free(p, (void *)stream, alloc->ctx);
    else (void)hipFree(p);
}
