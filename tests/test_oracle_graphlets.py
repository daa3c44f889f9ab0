"""Pins of the oracle's sampler, classifier, spanning-tree numbers and AGS (CPU only).

* class counts N_k (OEIS A001349; N_8 = 11117 is printed in the paper, Sec. 5.2)
* the class partition against networkx isomorphism over the graph atlas
* sigma_i against networkx's matrix-tree count, closed forms and sum_j sigma_ij
* t = sum_i c_i sigma_i and t_j = sum_i c_i sigma_ij over colourful induced
  subgraphs (the identity behind E[chi_i] = c_i sigma_i / t, Sec. 2.2)
* the sampler's law: each colourful copy with probability 1/t (Sec. 2.2), by a
  chi-square test with a fixed seed; shape-restricted sampling likewise
* AGS (Sec. 4.1) on the lollipop graph of the lower bound of Sec. 4.3
"""
from __future__ import annotations

import math
from collections import Counter, defaultdict

import networkx as nx
import numpy as np
import pytest
from scipy import stats

import graphgen as gg
import oracle as O
import brute


def code_of(H, order, k):
    idx = O.pair_index(k)
    c = 0
    for i in range(k):
        for j in range(i + 1, k):
            if H.has_edge(order[i], order[j]):
                c |= 1 << idx[(i, j)]
    return c


def atlas_connected(k):
    return [G for G in nx.graph_atlas_g() if G.number_of_nodes() == k and nx.is_connected(G)]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7])
def test_class_counts(k):
    assert O.num_classes(k) == [1, 1, 2, 6, 21, 112, 853][k - 1]


@pytest.mark.slow
def test_class_count_k8_printed_in_paper():
    # Sec. 5.2: 11117 distinct 8-graphlets
    assert O.num_classes(8) == 11117


@pytest.mark.parametrize("k", [4, 5, 6, 7])
def test_classify_partition_matches_isomorphism(k):
    graphs = atlas_connected(k)
    assert len(graphs) == O.num_classes(k)
    rng = np.random.default_rng(k)
    # host graph: disjoint union of every atlas graph, each with shuffled labels
    edges, verts = [], []
    base = 0
    for G in graphs:
        perm = rng.permutation(k)
        for a, b in G.edges():
            edges.append((base + perm[a], base + perm[b]))
        order = rng.permutation(k)
        verts.append([base + int(x) for x in order])
        base += k
    host = gg.csr_from_edges(base, np.array(edges, np.int64))
    code, cls = O.classify(host, k, np.array(verts, np.int32))
    assert sorted(cls.tolist()) == list(range(len(graphs)))   # a bijection
    # classes are ranked by canonical code, and a code's class is that of its canonical code
    cat = O.catalog_codes(k)
    assert np.all(np.diff(cat.astype(np.int64)) > 0)
    for c, q in zip(code, cls):
        assert cat[q] == O.canonical_code(int(c), k)


@pytest.mark.parametrize("k", [3, 4, 5, 6, 7])
def test_spanning_trees_match_networkx(k):
    for G in atlas_connected(k)[:300]:
        order = list(G.nodes())
        c = code_of(G, order, k)
        sig = O.spanning_trees(c, k)
        assert sig == round(nx.number_of_spanning_trees(G))
        assert int(O.spanning_trees_by_shape(c, k).sum()) == sig


def test_spanning_tree_closed_forms():
    for k in range(2, 9):
        Kk = nx.complete_graph(k)
        assert O.spanning_trees(code_of(Kk, list(range(k)), k), k) == k ** (k - 2)   # Cayley
        if k >= 3:
            Ck = nx.cycle_graph(k)
            assert O.spanning_trees(code_of(Ck, list(range(k)), k), k) == k
        P = nx.path_graph(k)
        assert O.spanning_trees(code_of(P, list(range(k)), k), k) == 1
    # sigma_ij of a star graph: one spanning tree, the star shape
    k = 6
    S = nx.star_graph(k - 1)
    by = O.spanning_trees_by_shape(code_of(S, list(range(k)), k), k)
    assert by.sum() == 1


@pytest.mark.parametrize("k", [3, 4, 5])
def test_totals_equal_sum_over_induced_graphlets(k):
    # t = sum_i c_i sigma_i and t_j = sum_i c_i sigma_ij (P9)
    g = gg.erdos_renyi(11, 22, seed=17 + k)
    colors = gg.colors(g.n, k, seed=40 + k)
    tab = O.Table(g, colors, k)
    t, tj = tab.totals()
    tot = 0
    totj = np.zeros(O.num_unrooted(k), np.int64)
    for vs, H in brute.colourful_graphlets(g, colors, k):
        c = code_of(H, list(vs), k)
        tot += O.spanning_trees(c, k)
        totj += O.spanning_trees_by_shape(c, k)
    assert t == tot
    assert tj == totj.tolist()


def _copy_of(verts, par):
    return frozenset((min(int(verts[i]), int(verts[par[i]])), max(int(verts[i]), int(verts[par[i]])))
                     for i in range(1, len(verts)))


def _colourful_copies(g, colors, k):
    out = []
    for vs, es in brute.subtrees(g, k):
        if len({int(colors[v]) for v in vs}) == k:
            out.append(frozenset(es))
    return out


@pytest.mark.parametrize("rooting", [O.ROOT_ZERO, O.ROOT_ALL])
def test_sampler_uniform_over_copies(rooting):
    # Sec. 2.2: every colourful k-treelet copy is drawn with probability 1/t
    g = gg.erdos_renyi(9, 16, seed=21)
    k = 4
    colors = gg.colors(g.n, k, seed=5)
    tab = O.Table(g, colors, k, rooting)
    copies = _colourful_copies(g, colors, k)
    t, _ = tab.totals()
    assert t == len(copies) > 10
    N = 40 * t
    verts, par = tab.sample(N, seed=123, stream=1)
    seen = Counter()
    for s in range(N):
        vs = verts[s]
        assert len(set(vs.tolist())) == k
        assert len({int(colors[v]) for v in vs}) == k
        if rooting == O.ROOT_ZERO:
            assert colors[vs[0]] == 0
        for i in range(1, k):
            assert g.neighbors(vs[par[s][i]]).tolist().count(vs[i]) == 1
        seen[_copy_of(vs, par[s])] += 1
    assert set(seen) <= set(copies)
    obs = np.array([seen[c] for c in copies])
    p = stats.chisquare(obs).pvalue
    assert p > 1e-3, p


def test_sampler_shape_restricted():
    # sample(T) of Sec. 4.1: copies of one unrooted shape, each with probability 1/t_j
    g = gg.erdos_renyi(9, 17, seed=2)
    k = 4
    colors = gg.colors(g.n, k, seed=8)
    tab = O.Table(g, colors, k)
    _, tj = tab.totals()
    for j in range(O.num_unrooted(k)):
        if tj[j] == 0:
            continue
        copies = []
        for vs, es in brute.subtrees(g, k):
            if len({int(colors[v]) for v in vs}) != k:
                continue
            adj = defaultdict(set)
            for a, b in es:
                adj[a].add(b)
                adj[b].add(a)
            s = min(brute.rooted_string(adj, r) for r in vs)
            rank = [O.shape_string(k, q) for q in range(O.num_shapes(k))].index(s)
            if O.shape_unrooted(k, rank) == j:
                copies.append(frozenset(es))
        assert len(copies) == tj[j]
        N = 40 * tj[j]
        verts, par = tab.sample(N, seed=9, stream=j, shape=j)
        seen = Counter(_copy_of(verts[s], par[s]) for s in range(N))
        assert set(seen) <= set(copies)
        obs = np.array([seen[c] for c in copies])
        if len(copies) > 1:
            assert stats.chisquare(obs).pvalue > 1e-3


def test_sampler_stream_is_indexed():
    g = gg.erdos_renyi(30, 70, seed=1)
    k = 5
    tab = O.Table(g, gg.colors(g.n, k, seed=2), k)
    v1, p1 = tab.sample(40, seed=77, stream=3)
    v2, p2 = tab.sample(25, seed=77, stream=3, first_index=15)
    assert np.array_equal(v1[15:], v2) and np.array_equal(p1[15:], p2)
    v3, _ = tab.sample(40, seed=77, stream=4)
    assert not np.array_equal(v1, v3)


def test_class_frequencies_follow_sigma():
    # E[chi_i] = c_i sigma_i / t (Sec. 2.2): class frequencies of uniform samples
    g = gg.erdos_renyi(12, 30, seed=6)
    k = 4
    colors = gg.colors(g.n, k, seed=12)
    tab = O.Table(g, colors, k)
    t, _ = tab.totals()
    expect = defaultdict(int)
    for vs, H in brute.colourful_graphlets(g, colors, k):
        c = code_of(H, list(vs), k)
        cls = O.classify(g, k, np.array([vs], np.int32))[1][0]
        expect[int(cls)] += O.spanning_trees(c, k)
    N = 20000
    verts, _ = tab.sample(N, seed=5)
    _, cls = O.classify(g, k, verts)
    obs = Counter(cls.tolist())
    keys = sorted(expect)
    assert set(obs) <= set(keys)
    f_obs = np.array([obs[i] for i in keys], float)
    f_exp = np.array([expect[i] * N / t for i in keys], float)
    assert stats.chisquare(f_obs, f_exp).pvalue > 1e-3


def _truth_by_class(g, colors, k):
    truth = Counter()
    for vs, H in brute.colourful_graphlets(g, colors, k):
        truth[int(O.classify(g, k, np.array([vs], np.int32))[1][0])] += 1
    return truth


def test_ags_covers_lollipop_classes():
    # Sec. 4.3's lollipop graph: AGS covers every class present, and its
    # estimates c_i / w_i are close to the colourful counts c_i
    k = 4
    g = gg.lollipop(14, 2)
    path_cls = int(O.classify(gg.path(4), 4, np.array([[0, 1, 2, 3]], np.int32))[1][0])
    for cseed in range(100):          # first colouring with a colourful induced path
        colors = gg.colors(g.n, k, seed=cseed)
        truth = _truth_by_class(g, colors, k)
        if truth[path_cls] > 0:
            break
    assert truth[path_cls] > 0
    tab = O.Table(g, colors, k)
    cbar = 200
    res = tab.ags(cbar=cbar, round_size=100, budget=400_000, seed=4, stream=0)
    for i, c in truth.items():
        assert res["hits"][i] >= cbar
        est = res["hits"][i] / res["w"][i]
        assert abs(est - c) <= 0.3 * c, (i, est, c)
    # replay is deterministic
    res2 = tab.ags(cbar=cbar, round_size=100, budget=400_000, seed=4, stream=0)
    assert np.array_equal(res["hits"], res2["hits"]) and np.array_equal(res["round_shapes"], res2["round_shapes"])


def test_ags_switches_away_from_covered_graphlets():
    # Sec. 4.1: a hub with many leaves plus a separate path. Uniform samples are
    # almost all stars; once the star graphlet is covered AGS switches to the
    # path treelet, whose copies span only the rare path graphlet.
    k = 4
    leaves, plen = 80, 9
    edges = [(0, i) for i in range(1, leaves + 1)]
    edges += [(leaves + 1 + i, leaves + 2 + i) for i in range(plen - 1)]
    g = gg.csr_from_edges(leaves + 1 + plen, np.array(edges, np.int64))
    path_cls = int(O.classify(gg.path(4), 4, np.array([[0, 1, 2, 3]], np.int32))[1][0])
    for cseed in range(200):
        colors = gg.colors(g.n, k, seed=cseed)
        truth = _truth_by_class(g, colors, k)
        if truth[path_cls] >= 2:
            break
    tab = O.Table(g, colors, k)
    cbar, budget = 100, 6000
    res = tab.ags(cbar=cbar, round_size=50, budget=budget, seed=11, stream=2)
    assert res["hits"][path_cls] >= cbar
    assert abs(res["hits"][path_cls] / res["w"][path_cls] - truth[path_cls]) <= 0.3 * truth[path_cls]
    n_used = int(res["n_j"].sum())
    verts, _ = tab.sample(n_used, seed=11, stream=2)
    _, cls = O.classify(g, k, verts)
    assert (cls == path_cls).sum() < cbar / 4
