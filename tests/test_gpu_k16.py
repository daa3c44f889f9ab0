"""GPU build for k up to 16 (sparse records keyed by DFS bitstring, Sec. 3.2)
against the sparse oracle, bit for bit: every level's offsets, keys and both
count words, and t.

Cases: k = 2..8 on random graphs under both rootings with tiny and default
term chunks (many chunks, one chunk); k = 9..12 on bounded-degree graphs and
a graph with a hub (long neighbour-sum records: the combine's binary-search
path); k = 16 on a sparse graph; the degenerate graphs (no vertex, isolated
vertices, no colourful treelet); a host graph (copied by the library); the
error paths; and counts at the 128-bit limit: a star whose k = 16 centre count
needs 136 bits (SCC_EOVERFLOW) while every level below stays exact, checked
against the closed form (products of colour class sizes).
"""
from __future__ import annotations

from math import prod

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from gpu_util import scc as _load_scc

pytestmark = pytest.mark.gpu


class _Lib:
    """The library, imported on first use (collection runs without a GPU)."""

    def __getattr__(self, name):
        return getattr(_load_scc(), name)


scc = _Lib()


def _tables_equal(gt, ot, k, what):
    for h in range(1, k + 1):
        go, gk, gl, gh = gt.export_level(h)
        oo, ok, ol, oh = ot.export_level(h)
        assert np.array_equal(go, oo), (what, h, "offsets")
        assert np.array_equal(gk, ok), (what, h, "keys")
        assert np.array_equal(gl, ol) and np.array_equal(gh, oh), (what, h, "counts")
    assert gt.total() == ot.total(), what


def _pair(g, colors, k, rooting, chunk_terms=0, host=False):
    graph = g if host else scc.DeviceGraph.from_graph(g)
    gt = scc.Table16(graph, colors, k, rooting=rooting, chunk_terms=chunk_terms)
    ot = O.Table16(g, colors, k, rooting)
    return gt, ot


def _sparse_graph(n, extra, seed):
    """A random tree on n vertices plus `extra` chords."""
    rng = np.random.default_rng(seed)
    edges = {(int(rng.integers(0, v)), v) for v in range(1, n)}
    while len(edges) < n - 1 + extra:
        a, b = sorted(int(x) for x in rng.choice(n, 2, replace=False))
        edges.add((a, b))
    return gg.csr_from_edges(n, np.array(sorted(edges), np.int64))


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("rooting", [O.ROOT_ZERO, O.ROOT_ALL])
def test_small_k_random_graphs(k, rooting):
    for name, g in (("er", gg.erdos_renyi(60, 150, seed=k)), ("cl", gg.chung_lu(120, 300, 2.2, 20, seed=k)),
                    ("lollipop", gg.lollipop(7, 4))):
        colors = gg.colors(g.n, k, seed=3 * k + rooting)
        for chunk in (0, 37):
            gt, ot = _pair(g, colors, k, rooting, chunk_terms=chunk)
            _tables_equal(gt, ot, k, f"{name} k={k} chunk={chunk}")
            if chunk:
                inf = gt.info()
                for h in range(2, k + 1):
                    assert inf.chunks[h] >= (2 if inf.terms[h] > chunk else 0), h


@pytest.mark.parametrize("k,n,extra,seed", [(9, 60, 20, 1), (10, 50, 15, 2), (11, 40, 10, 3), (12, 30, 8, 7)])
@pytest.mark.parametrize("rooting", [O.ROOT_ZERO, O.ROOT_ALL])
def test_k9_to_k12_sparse_graphs(k, n, extra, seed, rooting):
    g = _sparse_graph(n, extra, seed)
    colors = gg.colors(g.n, k, seed=seed + 40)
    gt, ot = _pair(g, colors, k, rooting, chunk_terms=4096)
    _tables_equal(gt, ot, k, f"k={k}")
    assert ot.total() > 0


def test_k10_hub():
    # a hub of degree 40 inside a sparse graph: long neighbour sums at the hub
    g0 = _sparse_graph(70, 10, 7)
    edges = [(int(v), int(u)) for v in range(g0.n) for u in g0.col_idx[g0.row_ptr[v]:g0.row_ptr[v + 1]] if v < u]
    edges += [(0, v) for v in range(30, 70) if (0, v) not in edges]
    g = gg.csr_from_edges(g0.n, np.array(sorted(set(edges)), np.int64))
    colors = gg.colors(g.n, 10, seed=9)
    gt, ot = _pair(g, colors, 10, O.ROOT_ALL)
    _tables_equal(gt, ot, 10, "hub")


def test_k16_sparse_graph():
    g = _sparse_graph(34, 4, 11)
    colors = (np.random.default_rng(5).permutation(g.n) % 16).astype(np.uint8)
    for rooting in (O.ROOT_ZERO, O.ROOT_ALL):
        gt, ot = _pair(g, colors, 16, rooting)
        _tables_equal(gt, ot, 16, f"k=16 rooting {rooting}")


def test_degenerate_graphs():
    # no vertex
    g = gg.csr_from_edges(0, np.zeros((0, 2), np.int64))
    t = scc.Table16(g, np.zeros(0, np.uint8), 5)
    assert t.total() == 0 and all(t.info().nnz[h] == 0 for h in range(1, 6))
    # isolated vertices around a path; a colouring with no colourful treelet
    g = gg.csr_from_edges(12, np.array([(2, 3), (3, 4), (4, 5), (5, 6)], np.int64))
    for colors in (gg.colors(12, 4, seed=2), np.zeros(12, np.uint8)):
        gt, ot = _pair(g, colors, 4, O.ROOT_ALL)
        _tables_equal(gt, ot, 4, "isolated")


def test_host_graph_copy():
    g = gg.erdos_renyi(80, 200, seed=3)
    colors = gg.colors(g.n, 9, seed=4)
    gt, ot = _pair(g, colors, 9, O.ROOT_ZERO, host=True)
    _tables_equal(gt, ot, 9, "host graph")


def test_invalid_inputs():
    g = gg.erdos_renyi(30, 60, seed=1)
    dg = scc.DeviceGraph.from_graph(g)
    colors = gg.colors(g.n, 5, seed=1)
    for k in (1, 17):
        with pytest.raises(scc.SccError) as e:
            scc.Table16(dg, colors, k)
        assert e.value.status == scc.EINVAL
    with pytest.raises(scc.SccError) as e:
        scc.Table16(dg, colors, 5, rooting=scc.ROOT_BALANCED)
    assert e.value.status == scc.EINVAL
    bad = colors.copy()
    bad[3] = 5
    with pytest.raises(scc.SccError) as e:
        scc.Table16(dg, bad, 5)
    assert e.value.status == scc.EINVAL
    # an asymmetric row: drop one direction of an edge
    ci = g.col_idx.copy()
    v = int(np.argmax(np.diff(g.row_ptr)))
    ci[g.row_ptr[v]] = ci[g.row_ptr[v] + 1] if g.row_ptr[v + 1] - g.row_ptr[v] > 1 else ci[g.row_ptr[v]]
    asym = gg.Graph(g.n, g.row_ptr.copy(), ci) if hasattr(gg, "Graph") else None
    if asym is not None:
        with pytest.raises(scc.SccError) as e:
            scc.Table16(scc.DeviceGraph.from_graph(asym), colors, 5)
        assert e.value.status == scc.EINVAL


def test_star_beyond_128_bits():
    # centre colour 0, leaf i colour 1 + i % 15: class sizes 546 and 547. The only
    # colourful 16-treelets are the stars around the centre, one for each choice
    # of a leaf of every colour: the centre's level-16 count and t are the product
    # of the 15 class sizes (about 2^136). A 128-bit build stops with
    # SCC_EOVERFLOW; the default builds again with 256-bit counts.
    d = 8192
    g = gg.star(d)
    colors = np.concatenate([[0], 1 + np.arange(d) % 15]).astype(np.uint8)
    sizes = np.bincount(colors[1:], minlength=16)
    want = prod(int(sizes[c]) for c in range(1, 16))
    assert want > 1 << 128
    dg = scc.DeviceGraph.from_graph(g)
    with pytest.raises(scc.SccError) as e:
        scc.Table16(dg, colors, 16, max_bits=128)
    assert e.value.status == scc.EOVERFLOW
    t = scc.Table16(dg, colors, 16)
    assert t.count_bits() == 256
    assert t.total() == want
    off, key, words = t.export_words(16)
    star = int("10" * 15, 2)
    got = {int(key[q]): O.words_int(words[q]) for q in range(off[0], off[1])}
    assert got == {(star << 16) | 0xffff: want}
    assert off[-1] == off[1]                      # zero-rooting: level 16 at the centre only
    # level 15 at a leaf: the leaf, then the centre with 13 more leaves
    off, key, words = t.export_words(15)
    leaf = 1
    cl = int(colors[leaf])
    for q in range(off[leaf], off[leaf + 1]):
        C = int(key[q]) & 0xffff
        others = [c for c in range(1, 16) if C >> c & 1 and c != cl]
        assert O.words_int(words[q]) == prod(int(sizes[c]) for c in others)


@pytest.mark.parametrize("k,rooting", [(5, O.ROOT_ALL), (9, O.ROOT_ZERO), (11, O.ROOT_ALL)])
def test_256_bit_build_equals_oracle(k, rooting):
    # the 256-bit kernels on graphs whose counts are small: every level equals the
    # oracle's (itself computed in 256 bits), word for word
    g = _sparse_graph(44, 12, 30 + k) if k > 8 else gg.erdos_renyi(80, 240, seed=k)
    colors = gg.colors(g.n, k, seed=k + 3)
    gt = scc.Table16(scc.DeviceGraph.from_graph(g), colors, k, rooting=rooting, max_bits=256, chunk_terms=500)
    ot = O.Table16(g, colors, k, rooting)
    assert gt.count_bits() == 256
    for h in range(1, k + 1):
        go, gk, gw = gt.export_words(h)
        oo, ok, ow = ot.export_words(h)
        assert np.array_equal(go, oo) and np.array_equal(gk, ok) and np.array_equal(gw, ow), h
    assert gt.total() == ot.total()
    with pytest.raises(scc.SccError) as e:
        gt.export_level(k)                        # two words cannot hold a 256-bit table's counts
    assert e.value.status == scc.EINVAL


def test_star_closed_form_beyond_64_bits():
    # k = 15, 4096 leaves coloured 1 + i % 14: the only colourful 15-treelets
    # are the 15-stars around the centre, so the centre's level-15 record is one
    # count, the product of the 14 class sizes (about 2^115), and so is t
    d, k = 4096, 15
    g = gg.star(d)
    colors = np.concatenate([[0], 1 + np.arange(d) % 14]).astype(np.uint8)
    sizes = np.bincount(colors[1:], minlength=k)
    want = prod(int(sizes[c]) for c in range(1, k))
    assert (1 << 64) < want < (1 << 128)
    t = scc.Table16(scc.DeviceGraph.from_graph(g), colors, k, rooting=scc.ROOT_ALL)
    off, key, lo, hi = t.export_level(k)
    star = int("10" * (k - 1), 2)
    cnt = {int(key[q]): int(lo[q]) | (int(hi[q]) << 64) for q in range(off[0], off[1])}
    assert cnt == {(star << 16) | ((1 << k) - 1): want}
    assert t.total() == want
    # a leaf's level-h counts: the leaf, then the centre with h-2 leaves
    off, key, lo, hi = t.export_level(5)
    leaf = 1
    path_star = int("1" + "10" * 3 + "0", 2)
    for q in range(off[leaf], off[leaf + 1]):
        assert int(key[q]) >> 16 == path_star
        C = int(key[q]) & 0xffff
        cl = int(colors[leaf])
        assert C & 1 and C >> cl & 1
        others = [c for c in range(1, k) if C >> c & 1 and c != cl]
        assert int(lo[q]) | (int(hi[q]) << 64) == prod(int(sizes[c]) for c in others)


def _ball(g, v, r):
    """Vertices within distance r of v (v first)."""
    seen = {v: 0}
    order = [v]
    frontier = [v]
    for d in range(r):
        nxt = []
        for x in frontier:
            for u in g.col_idx[g.row_ptr[x]:g.row_ptr[x + 1]]:
                u = int(u)
                if u not in seen:
                    seen[u] = d + 1
                    order.append(u)
                    nxt.append(u)
        frontier = nxt
    return order


def test_bench_workload_properties():
    # the k16 bench workload (Chung-Lu n = 65536, m = 131072, k = 10) at full size:
    # (1) zero-rooting and all rootings build identical levels 1..k-1 and the same t
    #     (each colourful copy has one colour-0 vertex, and k roots);
    # (2) a vertex's level-h record depends only on its ball of radius h-1, so for
    #     sampled vertices levels 2..4 equal the oracle's on that induced ball
    import torch
    g = gg.chung_lu(1 << 16, 1 << 17, 2.5, 40.0, seed=7)
    k = 10
    colors = gg.colors(g.n, k, seed=17)
    dg = scc.DeviceGraph.from_graph(g)
    tz = scc.Table16(dg, colors, k, rooting=scc.ROOT_ZERO)
    ta = scc.Table16(dg, colors, k, rooting=scc.ROOT_ALL)
    assert tz.total() == ta.total() > 0
    for h in range(1, k):
        a, b = tz.export_level(h, to_host=False), ta.export_level(h, to_host=False)
        assert all(torch.equal(x, y) for x, y in zip(a, b)), h
        del a, b
    levels = {h: tz.export_level(h) for h in (2, 3, 4)}
    rng = np.random.default_rng(3)
    deg = np.diff(g.row_ptr)
    picks = [int(np.argmax(deg))] + [int(x) for x in rng.choice(g.n, 12, replace=False)]
    for v in picks:
        ball = _ball(g, v, 3)
        pos = {u: i for i, u in enumerate(ball)}
        edges = [(pos[x], pos[int(u)]) for x in ball for u in g.col_idx[g.row_ptr[x]:g.row_ptr[x + 1]]
                 if int(u) in pos and pos[x] < pos[int(u)]]
        sub = gg.csr_from_edges(len(ball), np.array(edges, np.int64).reshape(-1, 2))
        ot = O.Table16(sub, colors[ball], k, O.ROOT_ALL)
        for h in (2, 3, 4):
            off, key, lo, hi = levels[h]
            oo, ok, ol, oh = ot.export_level(h)
            a, b = off[v], off[v + 1]
            assert np.array_equal(key[a:b], ok[oo[0]:oo[1]]), (v, h)
            assert np.array_equal(lo[a:b], ol[oo[0]:oo[1]]) and np.array_equal(hi[a:b], oh[oo[0]:oo[1]]), (v, h)
