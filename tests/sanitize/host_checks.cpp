// Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the
// library's host-side runtime: the treelet algebra and per-k lookup tables
// (treelets.cpp) with every index the kernels take from them checked against
// the staging layout, the serving arena's first-fit allocator under random
// admission and release, the allocator hooks of DevMem, and the exact small
// division of the combine. Exits 0 when every check holds and the sanitizers
// report nothing (they abort on the first finding).
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <random>
#include <vector>

#include "../../paper_2009_03052_amd/csrc/arena.hpp"
#include "../../paper_2009_03052_amd/csrc/scc_common.hpp"

static int fails = 0;
#define EXPECT(c)                                                        \
    do {                                                                 \
        if (!(c)) { std::fprintf(stderr, "failed: %s (line %d)\n", #c, __LINE__); fails++; } \
    } while (0)

static int binom(int n, int r) { if (r < 0 || r > n) return 0; int b = 1; for (int i = 1; i <= r; i++) b = b * (n - r + i) / i; return b; }

static void check_lut(int k)
{
    std::unique_ptr<DevLut> L(new DevLut);
    build_lut(k, L.get());
    static const int rooted[] = {0, 1, 1, 2, 4, 9, 20, 48, 115};
    static const int unrooted[] = {0, 1, 1, 1, 2, 3, 6, 11, 23};
    int keys = 0;
    for (int h = 1; h <= k; h++) {
        EXPECT(L->r[h] == rooted[h]);
        EXPECT(L->off[h] == keys);
        keys += L->r[h] * binom(k, h);
        EXPECT(L->W[h] == L->r[h] * binom(k - 1, h - 1));
        EXPECT(L->WS[h] == L->r[h] * binom(k - 1, h));
    }
    EXPECT(L->nkeys == keys);
    EXPECT(L->num_unr == unrooted[k]);
    for (int h = 2; h <= k; h++) {
        EXPECT(L->xoff[h] == L->xoff[h - 1] + L->W[h - 1]);
        EXPECT(L->soff[h] == L->soff[h - 1] + L->WS[h - 1]);
        for (int t = 0; t < L->r[h]; t++) {
            const int hp = L->dec_hp[h][t], hpp = h - hp;
            EXPECT(hp >= 1 && hpp >= 1);
            EXPECT(L->dec_a[h][t] < L->r[hp] && L->dec_b[h][t] < L->r[hpp]);
            EXPECT(L->dec_beta[h][t] >= 1 && L->dec_beta[h][t] <= h - 1);
        }
        // every output descriptor of level h: its terms stay inside the staged
        // own counts (levels < h) and neighbour sums (levels < h)
        for (int o = 0; o < L->W[h]; o++) {
            const uint64_t d = L->out[L->out_off[h] + o];
            const int xb = (int)(d & 0xffffu), sb = (int)((d >> 16) & 0xffffu), tb = (int)((d >> 32) & 0xffffu);
            const int ns = (int)((d >> 48) & 0xffu), beta = (int)((d >> 56) & 0x7fu);
            EXPECT(beta >= 1 && beta <= h - 1);
            EXPECT(tb + ns <= 2200);
            for (int i = 0; i < ns; i++) {
                const uint32_t xs = L->term_xs[tb + i];
                EXPECT(xb + (int)(xs & 0xffu) < L->xoff[h]);
                EXPECT(sb + (int)(xs >> 8) < L->soff[h]);
            }
            for (int c = 0; c < k; c++) EXPECT(L->out_key[c][L->out_off[h] + o] < L->nkeys);
        }
    }
    EXPECT(L->out_off[k] + L->W[k] <= 1400);
}

static void check_arena()
{
    std::mt19937_64 rng(7);
    Arena A;
    const int64_t cap = 1 << 24;
    A.reset(cap);
    std::map<int64_t, int64_t> live;   // offset -> bytes
    for (int it = 0; it < 200000; it++) {
        if (live.empty() || rng() % 3) {
            const int64_t b = 1 + (int64_t)(rng() % 200000);
            const int64_t off = A.alloc(b);
            if (off < 0) continue;
            EXPECT(off % 256 == 0 && off + Arena::round(b) <= cap);
            auto nx = live.lower_bound(off);
            if (nx != live.end()) EXPECT(off + Arena::round(b) <= nx->first);
            if (nx != live.begin()) { auto pv = std::prev(nx); EXPECT(pv->first + Arena::round(pv->second) <= off); }
            live[off] = b;
        } else {
            auto it2 = live.begin();
            std::advance(it2, (long)(rng() % live.size()));
            A.release(it2->first, it2->second);
            live.erase(it2);
        }
        int64_t used = 0;
        if (it % 1000 == 0) {
            for (auto &x : live) used += Arena::round(x.second);
            EXPECT(used == A.used());
        }
    }
    for (auto &x : live) A.release(x.first, x.second);
    EXPECT(A.used() == 0);
    EXPECT(A.alloc(cap) == 0);   // everything coalesced back into one range
}

static void *host_alloc(size_t b, void *, void *ctx) { ++*(int *)ctx; return std::malloc(b); }
static void host_free(void *p, void *, void *ctx) { --*(int *)ctx; std::free(p); }

static void check_devmem()
{
    int live = 0;
    scc_allocator al{host_alloc, host_free, &live};
    DevMem m;
    m.alloc = &al;
    std::vector<void *> ps;
    for (int i = 0; i < 100; i++) ps.push_back(m.get((size_t)i * 37));
    EXPECT(live == 100);
    for (void *p : ps) m.put(p);
    m.put(nullptr);
    EXPECT(live == 0);
}

static void check_division()
{
    std::mt19937_64 rng(3);
    for (int it = 0; it < 1000000; it++) {
        const uint32_t d = 1 + (uint32_t)(rng() % 8);
        const u128 q = mk128(rng(), rng() >> 3);
        EXPECT(div_exact_small(q * d, d) == q);
        EXPECT(div_small(q * d, d) == q);
        const uint64_t q64 = rng() >> 3;
        EXPECT(div_exact_small64(q64 * d, d) == q64);
    }
}

int main()
{
    for (int k = 1; k <= SCC_KMAX; k++) check_lut(k);
    check_arena();
    check_devmem();
    check_division();
    EXPECT(set_error(SCC_EINVAL, "x = %d", 5) == SCC_EINVAL);
    EXPECT(std::string(scc_last_error()) == "x = 5");
    if (fails) { std::fprintf(stderr, "%d checks failed\n", fails); return 1; }
    std::printf("host checks done\n");
    return 0;
}
