"""Pins of the oracle's round-skipping mode (balanced treelet decomposition and
direct star sampling, Sec. 3.3) against what the paper and mathematics fix.

* The lemma of the section: every unrooted k-treelet except the star has a
  rooting whose canonical decomposition is balanced (both parts of at least 2
  and at most k-2 nodes); the star has none. The designated rooting and its
  orbit (how many nodes of a copy give that rooting) are checked against
  rootings of explicit trees.
* With level k-1 skipped and level k kept at the designated rootings only, the
  per-shape totals of every non-star shape equal those of the zero-rooting
  table (itself pinned by brute force elsewhere); level k equals brute-force
  enumeration at the designated rootings; levels below k-1 are unchanged.
* Stars: sum_v binom(d_v, k-1) uncoloured copies, and the direct star sampler
  draws each (centre, leaf set) with equal probability.
* Shape-first uniform sampling draws every colourful non-star copy with
  probability 1/t, and shape-restricted sampling every copy of the shape with
  probability 1/t_j (chi-square against brute-force enumeration).
"""
from __future__ import annotations

import math
from collections import Counter, defaultdict

import numpy as np
import pytest
from scipy import stats

import graphgen as gg
import oracle as O
import brute


def _tree_from_string(s):
    """adjacency of the rooted tree with DFS bitstring s (root 0)."""
    adj = defaultdict(set)
    stack, nxt = [0], 1
    for ch in s:
        if ch == "1":
            adj[stack[-1]].add(nxt)
            adj[nxt].add(stack[-1])
            stack.append(nxt)
            nxt += 1
        else:
            stack.pop()
    adj[0]
    return adj


def _sizes_of_root_children(s):
    return [len(w) // 2 for w in brute.root_children_words(s)]


@pytest.mark.parametrize("k", [4, 5, 6, 7, 8])
def test_balanced_rootings_follow_the_lemma(k):
    strings = [O.shape_string(k, r) for r in range(O.num_shapes(k))]
    star = O.star_class(k)
    assert O.shape_unrooted(k, strings.index("10" * (k - 1))) == star
    for j in range(O.num_unrooted(k)):
        ranks = [r for r in range(O.num_shapes(k)) if O.shape_unrooted(k, r) == j]
        # balanced rootings: every root child has <= k-2 nodes and the largest >= 2
        bal = [r for r in ranks if max(_sizes_of_root_children(strings[r])) <= k - 2
               and max(_sizes_of_root_children(strings[r])) >= 2]
        if j == star:
            assert not bal and O.balanced_rank(k, j) == -1
            continue
        assert bal, f"non-star shape {j} without a balanced rooting"
        r = O.balanced_rank(k, j)
        assert r == min(bal)
        hp, _, _, _ = O.shape_decomp(k, r)
        assert 2 <= k - hp <= k - 2
        adj = _tree_from_string(strings[r])
        orbit = sum(brute.rooted_string(adj, x) == strings[r] for x in adj)
        assert O.balanced_orbit(k, j) == orbit


def _graphs():
    return [("er", gg.erdos_renyi(11, 22, seed=3)), ("cl", gg.chung_lu(40, 90, 2.2, 12, seed=4)),
            ("ba", gg.barabasi_albert(30, 2, seed=5)), ("lollipop", gg.lollipop(6, 5))]


@pytest.mark.parametrize("k", [4, 5, 6, 7])
@pytest.mark.parametrize("name,g", _graphs())
def test_balanced_totals_equal_zero_rooting(name, g, k):
    colors = gg.colors(g.n, k, seed=7 * k)
    zt = O.Table(g, colors, k, O.ROOT_ZERO)
    bt = O.Table(g, colors, k, O.ROOT_BALANCED)
    t0, tj0 = zt.totals()
    t1, tj1 = bt.totals()
    star = O.star_class(k)
    for j in range(O.num_unrooted(k)):
        assert tj1[j] == (0 if j == star else tj0[j]), (name, k, j)
    assert t1 == t0 - tj0[star]
    for h in range(1, k - 1):
        for a, b in zip(zt.export_level(h), bt.export_level(h)):
            assert np.array_equal(a, b), (name, k, h)
    assert bt.level_nnz(k - 1) == 0
    # level k: designated rootings only, at any vertex
    des = {O.balanced_rank(k, j) for j in range(O.num_unrooted(k)) if j != star}
    km = {}
    for r in range(O.num_shapes(k)):
        km[r] = O.key(k, k, r, (1 << k) - 1)
    keys = set(bt.export_level(k)[1].tolist())
    assert keys <= {km[r] for r in des}


@pytest.mark.parametrize("k", [4, 5])
def test_balanced_level_k_equals_brute_force(k):
    g = gg.erdos_renyi(10, 21, seed=11)
    colors = gg.colors(g.n, k, seed=12)
    bt = O.Table(g, colors, k, O.ROOT_BALANCED)
    ref = brute.treelet_counts(g, colors, k)[k]
    star = O.star_class(k)
    des = {O.shape_string(k, O.balanced_rank(k, j)) for j in range(O.num_unrooted(k)) if j != star}
    expect = {(v, s): c for (v, s, mask), c in ref.items() if s in des}
    got = {}
    off, key, lo, hi = bt.export_level(k)
    rank_of_key = {O.key(k, k, r, (1 << k) - 1): r for r in range(O.num_shapes(k))}
    for v in range(g.n):
        for q in range(off[v], off[v + 1]):
            got[(v, O.shape_string(k, rank_of_key[int(key[q])]))] = int(lo[q]) | (int(hi[q]) << 64)
    assert got == expect


@pytest.mark.parametrize("k", [4, 6, 8])
def test_star_count_closed_form(k):
    g = gg.chung_lu(300, 1500, 2.1, 60, seed=3)
    bt = O.Table(g, gg.colors(g.n, k, seed=1), k, O.ROOT_BALANCED)
    assert bt.star_count() == sum(math.comb(int(d), k - 1) for d in g.degrees())


def test_star_sampler_uniform_over_stars():
    g = gg.erdos_renyi(10, 24, seed=8)
    k = 4
    bt = O.Table(g, gg.colors(g.n, k, seed=2), k, O.ROOT_BALANCED)
    stars = []
    for v in range(g.n):
        nb = g.neighbors(v).tolist()
        for leaves in __import__("itertools").combinations(nb, k - 1):
            stars.append((v, frozenset(leaves)))
    assert len(stars) == bt.star_count() > 20
    N = 40 * len(stars)
    verts, par = bt.sample(N, seed=5, stream=2, shape=O.star_class(k))
    assert (par[:, 0] == -1).all() and (par[:, 1:] == 0).all()
    seen = Counter()
    for s in range(N):
        v, leaves = int(verts[s, 0]), verts[s, 1:].tolist()
        assert len(set(leaves)) == k - 1
        assert all(u in g.neighbors(v).tolist() for u in leaves)
        seen[(v, frozenset(leaves))] += 1
    assert set(seen) <= set(stars)
    obs = np.array([seen[c] for c in stars])
    assert stats.chisquare(obs).pvalue > 1e-3


def _copies_by_shape(g, colors, k):
    strings = [O.shape_string(k, q) for q in range(O.num_shapes(k))]
    out = defaultdict(list)
    for vs, es in brute.subtrees(g, k):
        if len({int(colors[v]) for v in vs}) != k:
            continue
        adj = defaultdict(set)
        for a, b in es:
            adj[a].add(b)
            adj[b].add(a)
        s = min(brute.rooted_string(adj, r) for r in vs)
        out[O.shape_unrooted(k, strings.index(s))].append(frozenset(es))
    return out


def _copy_of(verts, par):
    return frozenset((min(int(verts[i]), int(verts[par[i]])), max(int(verts[i]), int(verts[par[i]])))
                     for i in range(1, len(verts)))


def test_balanced_uniform_sampler_over_non_star_copies():
    g = gg.erdos_renyi(10, 22, seed=21)
    k = 4
    colors = gg.colors(g.n, k, seed=2)
    bt = O.Table(g, colors, k, O.ROOT_BALANCED)
    by = _copies_by_shape(g, colors, k)
    copies = [c for j, cs in by.items() if j != O.star_class(k) for c in cs]
    t, _ = bt.totals()
    assert t == len(copies) > 10
    N = 40 * t
    verts, par = bt.sample(N, seed=123, stream=1)
    seen = Counter(_copy_of(verts[s], par[s]) for s in range(N))
    assert set(seen) <= set(copies)
    assert stats.chisquare(np.array([seen[c] for c in copies])).pvalue > 1e-3


@pytest.mark.parametrize("k", [4, 5])
def test_balanced_shape_restricted_sampler(k):
    g = gg.erdos_renyi(11, 22, seed=9)
    colors = gg.colors(g.n, k, seed=10)
    bt = O.Table(g, colors, k, O.ROOT_BALANCED)
    _, tj = bt.totals()
    by = _copies_by_shape(g, colors, k)
    for j in range(O.num_unrooted(k)):
        if j == O.star_class(k) or tj[j] == 0:
            continue
        assert len(by[j]) == tj[j]
        N = 40 * tj[j]
        verts, par = bt.sample(N, seed=4, stream=j, shape=j)
        seen = Counter(_copy_of(verts[s], par[s]) for s in range(N))
        assert set(seen) <= set(by[j])
        if len(by[j]) > 1:
            assert stats.chisquare(np.array([seen[c] for c in by[j]])).pvalue > 1e-3


def test_balanced_mode_limits():
    g = gg.erdos_renyi(20, 40, seed=1)
    with pytest.raises(O.OracleError):
        O.Table(g, gg.colors(g.n, 3, seed=1), 3, O.ROOT_BALANCED)
    bt = O.Table(g, gg.colors(g.n, 5, seed=1), 5, O.ROOT_BALANCED)
    with pytest.raises(O.OracleError):
        bt.ags(cbar=10, round_size=10, budget=100, seed=1)
