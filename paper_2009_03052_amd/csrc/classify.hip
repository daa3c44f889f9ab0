// Graphlet classification (Sec. 4.4) and adaptive graphlet sampling (Sec. 4.1).
//
// The adjacency code of k ordered vertices is sum_{i<j} [v_i ~ v_j] 2^idx(i,j)
// with pairs numbered row by row; a graphlet's canonical code is the minimum
// code over all k! orders, and its class id is the rank of that code among the
// canonical codes of all connected k-vertex graphs.
//
// A per-k lookup table maps every code to its class. It is built on the GPU:
// each thread canonicalises one code by a branch-and-bound search over vertex
// orders (positions filled from the most significant row down; only vertices
// giving the smallest row survive, and of two interchangeable "twin" vertices
// only one is tried), flags the codes that are their own canonical form, and a
// scan of the flags ranks them.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "ags.hpp"
#include "sampler.hpp"

namespace {

__host__ __device__ inline int row_start(int p, int k) { return p * k - p * (p + 1) / 2; }
__host__ __device__ inline int pair_id(int i, int j, int k) { return row_start(i, k) + (j - i - 1); }

__host__ __device__ inline void code_to_adj(uint32_t code, int k, uint32_t *adj)
{
    for (int i = 0; i < k; i++) adj[i] = 0;
    for (int i = 0; i < k; i++)
        for (int j = i + 1; j < k; j++)
            if (code >> pair_id(i, j, k) & 1u) { adj[i] |= 1u << j; adj[j] |= 1u << i; }
}

__host__ __device__ inline bool adj_connected(const uint32_t *adj, int k)
{
    uint32_t seen = 1u, front = 1u;
    while (front) {
        uint32_t nf = 0;
        for (uint32_t f = front; f; f &= f - 1) nf |= adj[__builtin_ctz(f)];
        nf &= ~seen;
        seen |= nf;
        front = nf;
    }
    return seen == (1u << k) - 1u;
}

constexpr uint32_t NONE = 0xffffffffu;

// minimum adjacency code over all vertex orders (see file comment)
__host__ __device__ uint32_t canonical_min(uint32_t code, int k)
{
    uint32_t adj[SCC_KMAX];
    code_to_adj(code, k, adj);
    if (!adj_connected(adj, k)) return NONE;
    if (k == 1) return 0;
    uint32_t best = NONE;
    uint32_t cand[SCC_KMAX];   // remaining candidates at each position
    uint32_t at[SCC_KMAX];     // code with rows >= p fixed, per position
    int pos[SCC_KMAX];         // vertex at each position
    const uint32_t all = (1u << k) - 1u;
    uint32_t placed = 0;
    int p = k - 1;
    uint32_t cur = 0;
    bool enter = true;
    for (;;) {
        if (enter) {
            // rows of the unplaced vertices against positions p+1 .. k-1
            uint32_t m = 0xffffffffu, cset = 0;
            for (uint32_t f = all & ~placed; f; f &= f - 1) {
                const int x = __builtin_ctz(f);
                uint32_t r = 0;
                for (int q = p + 1; q < k; q++) r |= ((adj[x] >> pos[q]) & 1u) << (q - p - 1);
                if (r < m) { m = r; cset = 1u << x; }
                else if (r == m) cset |= 1u << x;
            }
            const int rs = row_start(p, k);
            const uint32_t code_p = cur | (m << rs);
            const int total = k * (k - 1) / 2;
            bool prune = false;
            if (best != NONE && rs < total) {
                const uint32_t a = code_p >> rs, b = best >> rs;
                prune = a > b;
            }
            if (!prune && p == 0) {
                if (code_p < best) best = code_p;
                prune = true;   // complete: go back up
            }
            if (!prune) {
                // one representative per class of twins (swapping twins is an automorphism)
                uint32_t keep = 0;
                for (uint32_t f = cset; f; f &= f - 1) {
                    const int x = __builtin_ctz(f);
                    bool twin = false;
                    for (uint32_t g = keep; g; g &= g - 1) {
                        const int y = __builtin_ctz(g);
                        if ((adj[x] & ~(1u << y)) == (adj[y] & ~(1u << x))) { twin = true; break; }
                    }
                    if (!twin) keep |= 1u << x;
                }
                cand[p] = keep;
                at[p] = code_p;
            } else {
                // move up to the nearest position with candidates left
                p++;
                while (p < k) {
                    placed &= ~(1u << pos[p]);
                    if (cand[p]) break;
                    p++;
                }
                if (p >= k) break;
            }
        }
        // take the next candidate at position p and descend
        const int x = __builtin_ctz(cand[p]);
        cand[p] &= cand[p] - 1;
        pos[p] = x;
        placed |= 1u << x;
        cur = at[p];
        p--;
        enter = true;
    }
    return best;
}

__global__ void k_canon(int k, uint64_t ncodes, uint32_t *canon, uint32_t *rep)
{
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncodes) return;
    const uint32_t m = canonical_min((uint32_t)c, k);
    canon[c] = m;
    rep[c] = (m == (uint32_t)c) ? 1u : 0u;
}

__global__ void k_class_lut(uint64_t ncodes, const uint32_t *canon, const uint32_t *rank_incl, uint16_t *lut,
                            uint32_t *cat)
{
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncodes) return;
    const uint32_t m = canon[c];
    lut[c] = m == NONE ? (uint16_t)0xffff : (uint16_t)(rank_incl[m] - 1u);
    if (m == (uint32_t)c) cat[rank_incl[c] - 1u] = (uint32_t)c;
}

// target in the sorted list col[lo, hi): halve the range down to CLS_WIN
// entries, then compare those entries, their loads issued together (one memory
// latency for the last four halvings of a binary search)
constexpr int CLS_WIN = 16;
__device__ inline bool in_sorted(const int32_t *col, int64_t lo, int64_t hi, int32_t target)
{
    while (hi - lo > CLS_WIN) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t w = col[mid];
        if (w == target) return true;
        if (w < target) lo = mid + 1; else hi = mid;
    }
    int32_t x[CLS_WIN];
#pragma unroll
    for (int q = 0; q < CLS_WIN; q++) x[q] = lo + q < hi ? col[lo + q] : -1;
    bool f = false;
#pragma unroll
    for (int q = 0; q < CLS_WIN; q++) f |= x[q] == target;
    return f;
}

// induced adjacency code of one sample (bit q for the q-th pair i < j) and its
// class through the lookup table; 0xffffffff for both when a vertex id is invalid.
// Every vertex's row bounds are read once; a pair searches the shorter row.
__device__ inline uint32_t classify_row(const GraphView &g, int k, const int32_t *row, const uint16_t *lut,
                                        uint32_t *code_out)
{
    int32_t vs[SCC_KMAX];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < SCC_KMAX; i++) {
        vs[i] = i < k ? row[i] : 0;
        ok = ok && (i >= k || (vs[i] >= 0 && vs[i] < g.n));
    }
    if (!ok) {
        *code_out = 0xffffffffu;
        return 0xffffffffu;
    }
    int64_t rb[SCC_KMAX], re[SCC_KMAX];
#pragma unroll
    for (int i = 0; i < SCC_KMAX; i++) {
        rb[i] = i < k ? g.row_ptr[vs[i]] : 0;
        re[i] = i < k ? g.row_ptr[vs[i] + 1] : 0;
    }
    // the pairs unrolled over SCC_KMAX vertices, so that the arrays stay in registers
    uint32_t code = 0;
    int q = 0;
#pragma unroll
    for (int i = 0; i < SCC_KMAX; i++)
#pragma unroll
        for (int j = i + 1; j < SCC_KMAX; j++) {
            if (j >= k) continue;
            const bool in_j = re[j] - rb[j] < re[i] - rb[i];
            if (in_j ? in_sorted(g.col_idx, rb[j], re[j], vs[i]) : in_sorted(g.col_idx, rb[i], re[i], vs[j]))
                code |= 1u << q;
            q++;
        }
    *code_out = code;
    const uint16_t c = lut[code];
    return c == 0xffff ? 0xffffffffu : (uint32_t)c;
}

__global__ void k_classify(GraphView g, int k, const int32_t *verts, int64_t n, const uint16_t *lut,
                           uint32_t *out_code, uint32_t *out_class)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t code;
    const uint32_t c = classify_row(g, k, verts + s * k, lut, &code);
    if (out_code) out_code[s] = code;
    out_class[s] = c;
}

// classes of the rows of a serving step (requests without a class output are skipped)
__global__ void k_serve_classify(const ServeClassArgs *args, const ServeChunk *ch, const int64_t *cend, int nch,
                                 int64_t total)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= total) return;
    int lo = 0, hi = nch - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cend[mid] > s) hi = mid; else lo = mid + 1;
    }
    const ServeChunk C = ch[lo];
    const ServeClassArgs &A = args[C.arg];
    if (!A.cls) return;
    const int64_t r = C.off + (s - (cend[lo] - C.count));
    uint32_t code;
    const uint32_t c = classify_row(A.g, A.k, A.verts + r * A.k, A.lut, &code);
    A.cls[r] = c;
    if (A.hist && c < A.nclass) atomicAdd(&A.hist[c], 1ull);
}

__global__ void k_hist(const uint32_t *cls, int64_t n, uint32_t nclass, unsigned long long *hist)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t c = cls[s];
    if (c < nclass) atomicAdd(&hist[c], 1ull);
}

// ---------------------------------------------------------------------------
// per-k class data, kept for the life of the process
// ---------------------------------------------------------------------------
struct ClassData {
    uint16_t *lut = nullptr;          // device, 2^(k(k-1)/2) entries
    std::vector<uint32_t> codes;      // canonical code of each class
    std::vector<int64_t> sigma;       // spanning trees
    std::vector<std::vector<int64_t>> sigma_ij;   // per class, computed on demand
    std::mutex sig_mu;
};

std::mutex g_cls_mu;
ClassData *g_cls[SCC_KMAX + 1];

scc_status ensure_classes(int k, hipStream_t st, ClassData **out)
{
    std::lock_guard<std::mutex> lk(g_cls_mu);
    if (g_cls[k]) { *out = g_cls[k]; return SCC_OK; }
    const int nb = k * (k - 1) / 2;
    const uint64_t ncodes = 1ull << nb;
    uint32_t *canon = nullptr, *rank = nullptr, *cat = nullptr;
    uint16_t *lut = nullptr;
    auto cleanup = [&]() { (void)hipFree(canon); (void)hipFree(rank); (void)hipFree(cat); };
    if (hipMalloc(&canon, ncodes * 4) != hipSuccess || hipMalloc(&rank, ncodes * 4) != hipSuccess ||
        hipMalloc(&lut, ncodes * 2) != hipSuccess || hipMalloc(&cat, 65536 * 4) != hipSuccess) {
        cleanup();
        (void)hipFree(lut);
        return set_error(SCC_ENOMEM, "class lookup table for k = %d", k);
    }
    const unsigned blocks = (unsigned)((ncodes + 255) / 256);
    hipLaunchKernelGGL(k_canon, dim3(blocks), dim3(256), 0, st, k, ncodes, canon, rank);
    // inclusive scan of the representative flags, in place
    scc_table tmp;
    tmp.stream = st;
    scc_status s = scan_u32(&tmp, rank, rank, (int64_t)ncodes);
    if (s) { cleanup(); (void)hipFree(lut); return s; }
    uint32_t nclass = 0;
    if (hipMemcpyAsync(&nclass, rank + (ncodes - 1), 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        cleanup(); (void)hipFree(lut);
        return set_error(SCC_EDEVICE, "class count");
    }
    hipLaunchKernelGGL(k_class_lut, dim3(blocks), dim3(256), 0, st, ncodes, canon, rank, lut, cat);
    ClassData *cd = new ClassData();
    cd->lut = lut;
    cd->codes.resize(nclass);
    hipError_t e = hipMemcpyAsync(cd->codes.data(), cat, nclass * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    cleanup();
    if (e != hipSuccess) { (void)hipFree(lut); delete cd; return set_error(SCC_EDEVICE, "class table: %s", hipGetErrorString(e)); }
    cd->sigma_ij.resize(nclass);
    g_cls[k] = cd;
    *out = cd;
    return SCC_OK;
}

// number of spanning trees: determinant of the reduced Laplacian modulo the
// prime 2^61 - 1 (the true value is below 8^6, so the residue is the value)
int64_t spanning_trees_host(uint32_t code, int k)
{
    if (k == 1) return 1;
    const uint64_t P = (1ull << 61) - 1;
    uint32_t adj[SCC_KMAX];
    code_to_adj(code, k, adj);
    const int m = k - 1;
    uint64_t A[SCC_KMAX][SCC_KMAX];
    for (int i = 0; i < m; i++)
        for (int j = 0; j < m; j++) {
            const int a = i + 1, b = j + 1;
            if (a == b) A[i][j] = (uint64_t)__builtin_popcount(adj[a]);
            else A[i][j] = (adj[a] >> b & 1u) ? P - 1 : 0;
        }
    auto mulm = [&](uint64_t x, uint64_t y) { return (uint64_t)(((u128)x * y) % P); };
    auto powm = [&](uint64_t x, uint64_t e) { uint64_t r = 1; while (e) { if (e & 1) r = mulm(r, x); x = mulm(x, x); e >>= 1; } return r; };
    uint64_t det = 1;
    for (int c = 0; c < m; c++) {
        int piv = -1;
        for (int r = c; r < m; r++) if (A[r][c]) { piv = r; break; }
        if (piv < 0) return 0;
        if (piv != c) { for (int j = 0; j < m; j++) std::swap(A[piv][j], A[c][j]); det = (P - det) % P; }
        det = mulm(det, A[c][c]);
        const uint64_t inv = powm(A[c][c], P - 2);
        for (int r = c + 1; r < m; r++) {
            if (!A[r][c]) continue;
            const uint64_t f = mulm(A[r][c], inv);
            for (int j = c; j < m; j++) A[r][j] = (A[r][j] + P - mulm(f, A[c][j])) % P;
        }
    }
    return (int64_t)det;
}

// unrooted shape of every labelled tree on k nodes, by edge code: the trees are
// the decodings of the k^(k-2) Pruefer sequences (Cayley); built once per k
const std::unordered_map<uint32_t, uint8_t> &tree_shapes(int k)
{
    static std::once_flag once[SCC_KMAX + 1];
    static std::unordered_map<uint32_t, uint8_t> maps[SCC_KMAX + 1];
    std::call_once(once[k], [k] {
        auto &m = maps[k];
        auto add = [&](const int *eu, const int *ev) {
            uint32_t code = 0, adj[SCC_KMAX] = {0};
            for (int e = 0; e < k - 1; e++) {
                code |= 1u << pair_id(std::min(eu[e], ev[e]), std::max(eu[e], ev[e]), k);
                adj[eu[e]] |= 1u << ev[e];
                adj[ev[e]] |= 1u << eu[e];
            }
            m.emplace(code, (uint8_t)tree_unrooted_id(k, adj));
        };
        if (k < 2) return;
        int64_t total = 1;
        for (int i = 0; i < k - 2; i++) total *= k;
        int seq[SCC_KMAX], eu[SCC_KMAX], ev[SCC_KMAX], deg[SCC_KMAX];
        for (int64_t x = 0; x < total; x++) {
            int64_t y = x;
            for (int i = 0; i < k - 2; i++) { seq[i] = (int)(y % k); y /= k; }
            for (int i = 0; i < k; i++) deg[i] = 1;
            for (int i = 0; i < k - 2; i++) deg[seq[i]]++;
            for (int i = 0; i < k - 2; i++) {
                int leaf = 0;
                while (deg[leaf] != 1) leaf++;
                eu[i] = leaf; ev[i] = seq[i];
                deg[leaf]--; deg[seq[i]]--;
            }
            int a = -1, b = -1;
            for (int i = 0; i < k; i++)
                if (deg[i] == 1) { if (a < 0) a = i; else b = i; }
            eu[k - 2] = a; ev[k - 2] = b;
            add(eu, ev);
        }
    });
    return maps[k];
}

// spanning trees of a graphlet by unrooted shape: a depth-first choice of k-1
// edges that never closes a cycle (every acyclic (k-1)-edge set on k vertices
// is a spanning tree); each tree's shape is looked up through its edge code
void spanning_trees_by_shape_host(uint32_t code, int k, int64_t *out)
{
    const int nu = unrooted_count(k);
    for (int j = 0; j < nu; j++) out[j] = 0;
    if (k == 1) { out[0] = 1; return; }
    const auto &shapes = tree_shapes(k);
    int eu[32], ev[32], ne = 0;
    for (int i = 0; i < k; i++)
        for (int j = i + 1; j < k; j++)
            if (code >> pair_id(i, j, k) & 1u) { eu[ne] = i; ev[ne] = j; ne++; }
    int comp[SCC_KMAX];
    for (int i = 0; i < k; i++) comp[i] = i;
    std::function<void(int, int, uint32_t)> rec = [&](int e, int chosen, uint32_t tcode) {
        if (chosen == k - 1) {
            out[shapes.at(tcode)]++;
            return;
        }
        if (ne - e < (k - 1) - chosen) return;
        // take edge e if it joins two components
        const int a = comp[eu[e]], b = comp[ev[e]];
        if (a != b) {
            int save[SCC_KMAX];
            memcpy(save, comp, sizeof save);
            for (int i = 0; i < k; i++) if (comp[i] == b) comp[i] = a;
            rec(e + 1, chosen + 1, tcode | (1u << pair_id(eu[e], ev[e], k)));
            memcpy(comp, save, sizeof save);
        }
        rec(e + 1, chosen, tcode);
    };
    rec(0, 0, 0);
}

}  // namespace

extern "C" scc_status scc_classify(const scc_table *T, const int32_t *verts, int64_t n, uint32_t *out_code,
                                   uint32_t *out_class, void *stream)
{
    if (!T) return set_error(SCC_EINVAL, "table NULL");
    if (n < 0) return set_error(SCC_EINVAL, "n < 0");
    if (n == 0) return SCC_OK;
    if (!verts || !out_class) return set_error(SCC_EINVAL, "NULL buffer");
    hipStream_t st = stream ? (hipStream_t)stream : T->stream;
    ClassData *cd;
    scc_status s = ensure_classes(T->k, st, &cd);
    if (s) return s;
    GraphView g{T->n, T->row_ptr, T->col_idx, T->colors};
    hipLaunchKernelGGL(k_classify, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, T->k, verts, n, cd->lut,
                       out_code, out_class);
    HIP_TRY(hipGetLastError());
    return SCC_OK;
}

extern "C" scc_status scc_catalog(int k, int64_t *num_classes, uint32_t *codes, int64_t *sigma, int64_t *sigma_ij,
                                  void *stream)
{
    if (k < 1 || k > SCC_KMAX) return set_error(SCC_EINVAL, "k out of range");
    ClassData *cd;
    scc_status s = ensure_classes(k, (hipStream_t)stream, &cd);
    if (s) return s;
    const int64_t nc = (int64_t)cd->codes.size();
    if (num_classes) *num_classes = nc;
    if (codes) memcpy(codes, cd->codes.data(), nc * 4);
    if (sigma)
        for (int64_t i = 0; i < nc; i++) sigma[i] = spanning_trees_host(cd->codes[i], k);
    if (sigma_ij) {
        const int nu = unrooted_count(k);
        std::vector<int> ids((size_t)nc);
        for (int64_t i = 0; i < nc; i++) ids[i] = (int)i;
        std::vector<const int64_t *> rows;
        class_sigma_rows(k, ids, rows);
        for (int64_t i = 0; i < nc; i++) memcpy(sigma_ij + i * nu, rows[i], (size_t)nu * 8);
    }
    return SCC_OK;
}

// Sec. 2.2: a uniform colourful k-treelet copy spans graphlet H_i with
// probability c_i sigma_i / t, so c_i ~= t (hits_i / n) / sigma_i; AGS gives
// c_i ~= hits_i / w_i; the copies in G are c_i / p_k.
extern "C" scc_status scc_estimate(const scc_table *T, const int64_t *hits, const double *w, int64_t n_samples,
                                   double p_k, double *out_colourful, double *out_count)
{
    if (!T || !hits) return set_error(SCC_EINVAL, "NULL argument");
    if (!w && n_samples <= 0) return set_error(SCC_EINVAL, "uniform estimates need n_samples > 0");
    const int k = T->k;
    ClassData *cd;
    scc_status s = ensure_classes(k, T->stream, &cd);
    if (s) return s;
    if (p_k <= 0) {
        p_k = 1.0;
        for (int i = 1; i <= k; i++) p_k *= (double)i / (double)k;
    }
    const double t = (double)T->t;
    for (size_t i = 0; i < cd->codes.size(); i++) {
        double c;
        if (w) c = w[i] > 0 ? (double)hits[i] / w[i] : 0.0;
        else c = t * ((double)hits[i] / (double)n_samples) / (double)spanning_trees_host(cd->codes[i], k);
        if (out_colourful) out_colourful[i] = c;
        if (out_count) out_count[i] = c / p_k;
    }
    return SCC_OK;
}

extern "C" void scc_release_caches(void)
{
    std::lock_guard<std::mutex> lk(g_cls_mu);
    for (int k = 0; k <= SCC_KMAX; k++) {
        if (g_cls[k]) { (void)hipFree(g_cls[k]->lut); delete g_cls[k]; g_cls[k] = nullptr; }
    }
}

void launch_serve_classify(const ServeClassArgs *args, const ServeChunk *ch, const int64_t *cend, int nch,
                           int64_t total, hipStream_t st)
{
    if (total <= 0 || nch <= 0) return;
    hipLaunchKernelGGL(k_serve_classify, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, args, ch, cend, nch,
                       total);
}

void class_sigma_rows(int k, const std::vector<int> &ids, std::vector<const int64_t *> &rows)
{
    ClassData *cd = g_cls[k];          // built by ensure_classes before any AGS state exists
    const int nu = unrooted_count(k);
    std::vector<int> todo;
    {
        std::lock_guard<std::mutex> lk(cd->sig_mu);
        for (int i : ids)
            if (cd->sigma_ij[i].empty()) todo.push_back(i);
    }
    if (!todo.empty()) {
        std::vector<std::vector<int64_t>> res(todo.size(), std::vector<int64_t>(nu));
        const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        const size_t nt = std::min<size_t>(hw, (todo.size() + 7) / 8);
        auto work = [&](size_t t) {
            for (size_t q = t; q < todo.size(); q += nt) spanning_trees_by_shape_host(cd->codes[todo[q]], k, res[q].data());
        };
        std::vector<std::thread> th;
        for (size_t t = 1; t < nt; t++) th.emplace_back(work, t);
        work(0);
        for (auto &x : th) x.join();
        std::lock_guard<std::mutex> lk(cd->sig_mu);
        for (size_t q = 0; q < todo.size(); q++)
            if (cd->sigma_ij[todo[q]].empty()) cd->sigma_ij[todo[q]] = std::move(res[q]);
    }
    std::lock_guard<std::mutex> lk(cd->sig_mu);
    rows.resize(ids.size());
    for (size_t q = 0; q < ids.size(); q++) rows[q] = cd->sigma_ij[ids[q]].data();
}

scc_status class_lut(int k, hipStream_t st, const uint16_t **lut, int *num_classes)
{
    ClassData *cd;
    scc_status s = ensure_classes(k, st, &cd);
    if (s) return s;
    *lut = cd->lut;
    if (num_classes) *num_classes = (int)cd->codes.size();
    return SCC_OK;
}

scc_status AgsState::init(const scc_table *T, int64_t cbar_, hipStream_t st)
{
    k = T->k;
    ClassData *cd;
    scc_status s = ensure_classes(k, st, &cd);
    if (s) return s;
    codes = cd->codes;
    S = (int)codes.size();
    NS = T->hlut.num_unr;
    cbar = cbar_;
    c.assign(S, 0); nj.assign(NS, 0); w.assign(S, 0.0); tjd.assign(NS, 0.0);
    cov.assign(S, 0); sig_ok.assign(S, 0); sig.assign(S, nullptr);
    shapes.clear();
    drawn = 0; ncov = 0; j = -1;
    for (int q = 0; q < NS; q++) tjd[q] = (double)T->tj[q];
    for (int q = 0; q < NS; q++)
        if (T->tj[q] > 0 && (j < 0 || T->tj[q] > T->tj[j])) j = q;
    if (j < 0) return set_error(SCC_EEMPTY, "no colourful %d-treelet", k);
    return SCC_OK;
}

void AgsState::add_round(int64_t n, const unsigned long long *hh)
{
    shapes.push_back(j);
    drawn += n;
    nj[j] += n;
    std::vector<int> fresh;
    for (int i = 0; i < S; i++) {
        if (!hh[i]) continue;
        c[i] += (int64_t)hh[i];
        if (!sig_ok[i]) { fresh.push_back(i); sig_ok[i] = 1; }
    }
    if (!fresh.empty()) {
        std::vector<const int64_t *> rows;
        class_sigma_rows(k, fresh, rows);
        for (size_t q = 0; q < fresh.size(); q++) sig[fresh[q]] = rows[q];
    }
    // Algorithm AGS tests the class each sample falls in: once its count has
    // reached cbar it is (or stays) covered and the shape is chosen again. A
    // round makes that test for every class it hit.
    bool reselect = false;
    for (int i = 0; i < S; i++) {
        if (!hh[i] || c[i] < cbar) continue;
        reselect = true;
        if (!cov[i]) { cov[i] = 1; ncov++; }
    }
    if (!reselect || ncov >= S) return;
    // w_i = sum_j n_j sigma_ij / t_j over covered classes, then the shape that
    // minimises (1/t_j) sum_{i covered} sigma_ij c_i / w_i; a score within a
    // relative 2^-40 of the best so far is a tie, and ties go to the smaller j
    // (exactly equal rationals are not split by rounding)
    for (int i = 0; i < S; i++) {
        if (!cov[i]) continue;
        double acc = 0.0;
        for (int q = 0; q < NS; q++)
            if (tjd[q] > 0) acc += (double)nj[q] * (double)sig[i][q] / tjd[q];
        w[i] = acc;
    }
    int best = -1;
    double bv = 0.0;
    for (int q = 0; q < NS; q++) {
        if (!(tjd[q] > 0)) continue;
        double acc = 0.0;
        for (int i = 0; i < S; i++)
            if (cov[i]) acc += (double)sig[i][q] * (double)c[i] / w[i];
        acc /= tjd[q];
        if (best < 0 || acc < bv * (1.0 - 0x1p-40)) { best = q; bv = acc; }
    }
    j = best;
}

void AgsState::result(int64_t *hits, double *w_out, int64_t *n_j) const
{
    for (int i = 0; i < S; i++) {
        double acc = 0.0;
        if (sig_ok[i])
            for (int q = 0; q < NS; q++)
                if (tjd[q] > 0) acc += (double)nj[q] * (double)sig[i][q] / tjd[q];
        hits[i] = c[i];
        w_out[i] = acc;
    }
    for (int q = 0; q < NS; q++) n_j[q] = nj[q];
}

extern "C" scc_status scc_ags(const scc_table *tc, int64_t cbar, int64_t round_size, int64_t budget, uint64_t seed,
                              uint64_t stream_id, int64_t *hits, double *w_out, int64_t *n_j, int32_t *round_shapes,
                              int64_t *n_rounds, void *stream)
{
    scc_table *T = const_cast<scc_table *>(tc);
    if (!T || !hits || !w_out || !n_j || !n_rounds) return set_error(SCC_EINVAL, "NULL argument");
    if (cbar < 1 || round_size < 1 || budget < 0) return set_error(SCC_EINVAL, "bad AGS parameters");
    if (T->rooting == SCC_ROOT_BALANCED)
        return set_error(SCC_EINVAL, "AGS needs zero-rooting or all rootings (round skipping drops stars from t_j)");
    const int k = T->k;
    hipStream_t st = stream ? (hipStream_t)stream : T->stream;
    AgsState A;
    scc_status s = A.init(T, cbar, st);
    if (s) return s;
    const int S = A.S;
    int32_t *dv = (int32_t *)T->mem.get((size_t)round_size * k * 4);
    int8_t *dp = (int8_t *)T->mem.get((size_t)round_size * k);
    uint32_t *dc = (uint32_t *)T->mem.get((size_t)round_size * 4);
    unsigned long long *dh = (unsigned long long *)T->mem.get((size_t)S * 8);
    std::vector<unsigned long long> hh(S);
    auto done = [&](scc_status r) { T->mem.put(dv); T->mem.put(dp); T->mem.put(dc); T->mem.put(dh); return r; };
    if (!dv || !dp || !dc || !dh) return done(set_error(SCC_ENOMEM, "AGS buffers"));
    while (!A.covered() && A.drawn + round_size <= budget) {
        s = scc_sample(T, A.j, round_size, seed, stream_id, (uint64_t)A.drawn, dv, dp, st);
        if (s) return done(s);
        s = scc_classify(T, dv, round_size, nullptr, dc, st);
        if (s) return done(s);
        if (hipMemsetAsync(dh, 0, (size_t)S * 8, st) != hipSuccess) return done(set_error(SCC_EDEVICE, "AGS memset"));
        hipLaunchKernelGGL(k_hist, dim3((unsigned)((round_size + 255) / 256)), dim3(256), 0, st, dc, round_size, (uint32_t)S, dh);
        if (hipMemcpyAsync(hh.data(), dh, (size_t)S * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return done(set_error(SCC_EDEVICE, "AGS histogram"));
        A.add_round(round_size, hh.data());
    }
    A.result(hits, w_out, n_j);
    if (round_shapes)
        for (size_t r = 0; r < A.shapes.size(); r++) round_shapes[r] = A.shapes[r];
    *n_rounds = (int64_t)A.shapes.size();
    return done(SCC_OK);
}
