"""Seeded synthetic inputs: simple undirected graphs in CSR form and colourings.

This module holds no counting arithmetic. It only produces inputs: a simple,
symmetric, row-sorted CSR (``row_ptr`` int64[n+1], ``col_idx`` int32[2m]) and a
colour vector ``colors`` uint8[n] with values in [0, k). Both the oracle and the
GPU library are fed from here, so the two sides always see identical inputs.

Generators (each draws from ``numpy.random.Generator(PCG64(seed))``):

* ``erdos_renyi(n, m, seed)``   -- G(n, m): uniform endpoint pairs, loops and
  duplicates rejected, until m distinct edges exist.
* ``chung_lu(n, m, gamma, wmax, seed)`` -- heavy-tailed expected-degree graph:
  weights w_i = wmax * (1 + i/i0)^(-1/(gamma-1)) with i0 chosen so that
  sum(w) = 2m; endpoints drawn proportionally to w until m distinct non-loop
  edges exist; vertices relabelled by a seeded random permutation.
* ``barabasi_albert(n, m0, seed)`` -- linear-time preferential attachment
  (Batagelj and Brandes, 2005): each new vertex links to m0 earlier ones chosen
  with probability proportional to degree.
* ``colors(n, k, seed)`` -- independent uniform colours in [0, k) (the colouring
  of colour coding, Section 2 of the paper).

Small deterministic graphs for tests: ``path``, ``cycle``, ``star``,
``complete``, ``lollipop`` (a clique with a dangling path, the adversarial
graph of the sampling lower bound in Section 4.3).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "Graph", "csr_from_edges", "erdos_renyi", "chung_lu", "barabasi_albert",
    "colors", "path", "cycle", "star", "complete", "lollipop", "from_networkx",
    "describe",
]


class Graph:
    """A simple undirected graph as a symmetric CSR with sorted rows."""

    __slots__ = ("n", "row_ptr", "col_idx")

    def __init__(self, n: int, row_ptr: np.ndarray, col_idx: np.ndarray):
        self.n = int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def edges(self) -> np.ndarray:
        """Undirected edge list (u < v), int64[m, 2]."""
        deg = self.degrees()
        src = np.repeat(np.arange(self.n, dtype=np.int64), deg)
        dst = self.col_idx.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)

    def neighbors(self, v: int) -> np.ndarray:
        return self.col_idx[self.row_ptr[v]:self.row_ptr[v + 1]]


def csr_from_edges(n: int, edges: np.ndarray) -> Graph:
    """Build the symmetric sorted CSR of an undirected edge list.

    Loops are dropped and duplicate edges merged, so the result is simple.
    """
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if e.size:
        u = np.minimum(e[:, 0], e[:, 1])
        v = np.maximum(e[:, 0], e[:, 1])
        keep = u != v
        key = np.unique(u[keep] * n + v[keep])
        u = key // n
        v = key % n
        # both directions; the keys are distinct, so sorting them orders the arcs
        arcs = np.sort(np.concatenate([u * n + v, v * n + u]))
        src = arcs // n
        dst = arcs % n
    else:
        src = np.zeros(0, np.int64)
        dst = np.zeros(0, np.int64)
    counts = np.bincount(src, minlength=n) if src.size else np.zeros(n, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n, row_ptr, dst.astype(np.int32))


def _first_occurrences(x: np.ndarray) -> np.ndarray:
    """Ascending positions of the first occurrence of each distinct value of x
    (what np.unique(x, return_index=True) gives, sorted), with a multi-threaded
    stable sort."""
    import torch
    sv, perm = torch.sort(torch.from_numpy(np.ascontiguousarray(x)), stable=True)
    head = torch.ones(sv.shape[0], dtype=torch.bool)
    if sv.shape[0] > 1:
        head[1:] = sv[1:] != sv[:-1]
    return np.sort(perm[head].numpy())


def _distinct_edges(n: int, m: int, draw, max_rounds: int = 64) -> np.ndarray:
    """Draw endpoint pairs with ``draw(count)`` until m distinct non-loop edges exist.

    Pairs are kept in the order they were drawn (the first m distinct ones).
    """
    keys = np.zeros(0, dtype=np.int64)
    need = m
    for _ in range(max_rounds):
        batch = max(int(need * 1.2) + 1024, 1024)
        a, b = draw(batch)
        lo = np.minimum(a, b)
        hi = np.maximum(a, b)
        ok = lo != hi
        new = lo[ok] * n + hi[ok]
        allk = np.concatenate([keys, new])
        keys = allk[_first_occurrences(allk)]
        if keys.shape[0] >= m:
            keys = keys[:m]
            break
        need = m - keys.shape[0]
    else:
        raise RuntimeError("could not draw enough distinct edges")
    return np.stack([keys // n, keys % n], axis=1)


def erdos_renyi(n: int, m: int, seed: int) -> Graph:
    """G(n, m) with uniformly drawn endpoint pairs."""
    if m > n * (n - 1) // 2:
        raise ValueError("m exceeds the number of vertex pairs")
    rng = np.random.Generator(np.random.PCG64(seed))

    def draw(c):
        return rng.integers(0, n, c, dtype=np.int64), rng.integers(0, n, c, dtype=np.int64)

    return csr_from_edges(n, _distinct_edges(n, m, draw))


def chung_lu_weights(n: int, m: int, gamma: float, wmax: float) -> np.ndarray:
    """w_i = wmax * (1 + i/i0)^(-1/(gamma-1)), with i0 solved so that sum(w) = 2m."""
    alpha = 1.0 / (gamma - 1.0)
    i = np.arange(n, dtype=np.float64)

    def total(i0):
        return float(np.sum(wmax * np.power(1.0 + i / i0, -alpha)))

    lo, hi = 1e-6, float(n) * 1e3
    if total(lo) > 2 * m or total(hi) < 2 * m:
        raise ValueError("no i0 gives the requested edge count")
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        if mid == lo or mid == hi:
            break   # adjacent doubles: later steps change nothing
        if total(mid) < 2 * m:
            lo = mid
        else:
            hi = mid
    return wmax * np.power(1.0 + i / hi, -alpha)


def _search_right(cdf: np.ndarray, x: np.ndarray) -> np.ndarray:
    """np.searchsorted(cdf, x, side="right"), multi-threaded."""
    import torch
    return torch.searchsorted(torch.from_numpy(cdf), torch.from_numpy(x), right=True).numpy().astype(np.int64)


def chung_lu(n: int, m: int, gamma: float, wmax: float, seed: int) -> Graph:
    """Heavy-tailed Chung--Lu graph with m distinct edges and relabelled vertices."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = chung_lu_weights(n, m, gamma, wmax)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]

    def draw(c):
        a = _search_right(cdf, rng.random(c))
        b = _search_right(cdf, rng.random(c))
        np.minimum(a, n - 1, out=a)
        np.minimum(b, n - 1, out=b)
        return a.astype(np.int64), b.astype(np.int64)

    e = _distinct_edges(n, m, draw)
    perm = rng.permutation(n).astype(np.int64)
    return csr_from_edges(n, perm[e])


def barabasi_albert(n: int, m0: int, seed: int) -> Graph:
    """Preferential attachment in linear time (Batagelj--Brandes, 2005)."""
    if n <= m0:
        raise ValueError("n must exceed m0")
    rng = np.random.Generator(np.random.PCG64(seed))
    # The endpoint list M holds every edge end once; a uniform entry of M is a
    # vertex drawn proportionally to its degree.
    M = np.zeros(2 * n * m0, dtype=np.int64)
    for v in range(n):
        for i in range(m0):
            M[2 * (v * m0 + i)] = v
            r = int(rng.integers(0, 2 * (v * m0 + i) + 1))
            M[2 * (v * m0 + i) + 1] = M[r]
    e = M.reshape(-1, 2)
    return csr_from_edges(n, e)


def colors(n: int, k: int, seed: int) -> np.ndarray:
    """Independent uniform colours in [0, k) as uint8."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, k, n, dtype=np.int64).astype(np.uint8)


def path(n: int) -> Graph:
    return csr_from_edges(n, np.array([(i, i + 1) for i in range(n - 1)], dtype=np.int64))


def cycle(n: int) -> Graph:
    return csr_from_edges(n, np.array([(i, (i + 1) % n) for i in range(n)], dtype=np.int64))


def star(leaves: int) -> Graph:
    """Vertex 0 is the centre."""
    return csr_from_edges(leaves + 1, np.array([(0, i) for i in range(1, leaves + 1)], dtype=np.int64))


def complete(n: int) -> Graph:
    return csr_from_edges(n, np.array([(i, j) for i in range(n) for j in range(i + 1, n)], dtype=np.int64))


def lollipop(clique: int, tail: int) -> Graph:
    """Clique on vertices [0, clique) plus a path of ``tail`` vertices hanging off vertex clique-1."""
    e = [(i, j) for i in range(clique) for j in range(i + 1, clique)]
    prev = clique - 1
    for t in range(tail):
        e.append((prev, clique + t))
        prev = clique + t
    return csr_from_edges(clique + tail, np.array(e, dtype=np.int64))


def two_hubs(d: int = 1 << 15, shared: int = 1 << 13, n_mid: int = 48, mid_deg: int = 150, seed: int = 5) -> Graph:
    """Two hubs of degree d over a path of 2d - shared leaves (the hubs share
    `shared` of them), plus n_mid vertices of degree mid_deg, each adjacent to
    mid_deg - 2 random leaves and to both hubs. The hubs take the two largest
    ids, so they come last in every row that holds them."""
    rng = np.random.default_rng(seed)
    L = 2 * d - shared
    A, B = L + n_mid, L + n_mid + 1
    e = [np.stack([np.arange(L - 1), np.arange(1, L)], 1),
         np.stack([np.full(d, A), np.arange(d)], 1),
         np.stack([np.full(d, B), np.arange(L - d, L)], 1)]
    for m in range(L, L + n_mid):
        nb = rng.choice(L, mid_deg - 2, replace=False)
        e.append(np.stack([np.full(nb.size, m), nb], 1))
        e.append(np.array([[m, A], [m, B]]))
    return csr_from_edges(L + n_mid + 2, np.concatenate(e).astype(np.int64))


def from_networkx(g) -> Graph:
    nodes = sorted(g.nodes())
    idx = {v: i for i, v in enumerate(nodes)}
    e = np.array([(idx[a], idx[b]) for a, b in g.edges()], dtype=np.int64).reshape(-1, 2)
    return csr_from_edges(len(nodes), e)


def describe(g: Graph) -> dict:
    """Realised size and degree statistics, for logs."""
    d = g.degrees()
    hist = np.bincount(np.minimum(np.floor(np.log2(np.maximum(d, 1))).astype(np.int64), 31))
    return {"n": g.n, "m": g.m, "d_max": int(d.max()) if g.n else 0,
            "d_mean": float(d.mean()) if g.n else 0.0,
            "log2_degree_hist": hist.tolist()}
