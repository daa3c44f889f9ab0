"""Pins of the oracle against what the paper and mathematics fix (CPU only).

Each test names the passage or fact it pins. None of them retypes the oracle's
formulas: they compare against brute-force enumeration from the definition, a
second algorithm (the per-edge pair join), exact identities over all
colourings, closed forms, numbers printed in the paper or in OEIS, and library
routines (numpy's Philox, networkx).
"""
from __future__ import annotations

import itertools
import math
from collections import defaultdict

import networkx as nx
import numpy as np
import pytest

import graphgen as gg
import oracle as O
import brute


def key_map(k):
    """oracle key -> (h, rank, mask), built through the oracle's key function."""
    m = {}
    for h in range(1, k + 1):
        for r in range(O.num_shapes(h)):
            for mask in range(1 << k):
                if bin(mask).count("1") == h:
                    m[O.key(k, h, r, mask)] = (h, r, mask)
    return m


def table_as_strings(tab, h):
    km = key_map(tab.k)
    out = {}
    for (v, key), c in tab.level_dict(h).items():
        hh, r, mask = km[key]
        assert hh == h
        out[(v, O.shape_string(h, r), mask)] = c
    return out


def small_graphs():
    out = [
        ("path6", gg.path(6)), ("cycle6", gg.cycle(6)), ("star5", gg.star(5)),
        ("K5", gg.complete(5)), ("lollipop", gg.lollipop(4, 3)),
    ]
    for s in range(4):
        out.append((f"er{s}", gg.erdos_renyi(9, 14, seed=100 + s)))
    out.append(("ba", gg.barabasi_albert(10, 2, seed=7)))
    return out


# --------------------------------------------------------------------------
# P1, P2, P3: treelet algebra
# --------------------------------------------------------------------------

def test_rooted_shape_counts_otter():
    # OEIS A000081, rooted trees on h nodes (the paper cites Otter for these counts)
    assert [O.num_shapes(h) for h in range(1, 9)] == [1, 1, 2, 4, 9, 20, 48, 115]


def test_unrooted_shape_counts():
    # OEIS A000055, free trees on h nodes
    assert [O.num_unrooted(h) for h in range(1, 9)] == [1, 1, 1, 2, 3, 6, 11, 23]


def test_key_space_1991():
    # Sec. 3.3: 1991 coloured rooted treelets on at most 8 nodes (11-bit ITE)
    assert O.num_keys(8) == 1991
    assert [O.num_keys(k) for k in range(4, 9)] == [22, 64, 195, 615, 1991]


def test_example_figure_encoding():
    # Sec. 3.2, example figure: root coloured 3 with children 1 (children 2, 7)
    # and 5 encodes as s_T = 11010010 and s_C = 10101110.
    adj = {3: {1, 5}, 1: {3, 2, 7}, 2: {1}, 7: {1}, 5: {3}}
    assert brute.rooted_string(adj, 3) == "11010010"
    assert "11010010" in [O.shape_string(5, r) for r in range(O.num_shapes(5))]
    # the oracle's DP on exactly this tree, coloured as in the figure, with k = 8
    n = 8
    edges = np.array([(3, 1), (3, 5), (1, 2), (1, 7)], dtype=np.int64)
    g = gg.csr_from_edges(n, edges)
    colors = np.arange(n, dtype=np.uint8)      # vertex i has colour i
    tab = O.Table(g, colors, 8, O.ROOT_ALL)
    lev = table_as_strings(tab, 5)
    mask = int("10101110", 2)
    assert lev[(3, "11010010", mask)] == 1
    # the merge of Sec. 3.2 is 1, s_T'', 0, s_T' with T'' the first child
    r = [O.shape_string(5, q) for q in range(O.num_shapes(5))].index("11010010")
    hp, a, b, beta = O.shape_decomp(5, r)
    assert (hp, O.shape_string(hp, a), O.shape_string(5 - hp, b), beta) == (2, "10", "1010", 1)


def test_shape_strings_are_canonical_and_complete():
    # every rooted tree on h <= 7 nodes (networkx's nonisomorphic trees, all rootings)
    for h in range(2, 8):
        strings = set()
        for t in nx.nonisomorphic_trees(h):
            adj = {v: set(t[v]) for v in t}
            for r in t:
                strings.add(brute.rooted_string(adj, r))
        ours = [O.shape_string(h, q) for q in range(O.num_shapes(h))]
        assert sorted(ours) == ours          # ranks follow ascending strings
        assert set(ours) == strings


def test_beta_and_automorphisms_cayley():
    # sum over rooted shapes of h!/|Aut| = h^(h-1) labelled rooted trees (Cayley)
    for h in range(1, 9):
        tot = sum(math.factorial(h) // brute.aut_rooted(O.shape_string(h, r)) for r in range(O.num_shapes(h)))
        assert tot == h ** (h - 1)
    # beta_T equals the multiplicity of the first child word
    for h in range(2, 9):
        for r in range(O.num_shapes(h)):
            s = O.shape_string(h, r)
            words = brute.root_children_words(s)
            hp, a, b, beta = O.shape_decomp(h, r)
            assert beta == words.count(words[0])
            assert O.shape_string(h - hp, b) == words[0][1:-1]
            assert O.shape_string(hp, a) == "".join(words[1:])


def test_unrooted_classes_match_free_trees():
    for h in range(2, 9):
        groups = defaultdict(set)
        for r in range(O.num_shapes(h)):
            groups[O.shape_unrooted(h, r)].add(O.shape_string(h, r))
        trees = list(nx.nonisomorphic_trees(h))
        expect = []
        for t in trees:
            adj = {v: set(t[v]) for v in t}
            expect.append({brute.rooted_string(adj, r) for r in t})
        assert sorted(map(sorted, groups.values())) == sorted(map(sorted, expect))
        # ids ascend with the smallest rooted rank of the class
        mins = [min(O.shape_string(h, r) for r in range(O.num_shapes(h)) if O.shape_unrooted(h, r) == j)
                for j in range(O.num_unrooted(h))]
        assert mins == sorted(mins)


# --------------------------------------------------------------------------
# P5: DP equals the definition; and equals the pair join of Sec. 3.1
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name,g", small_graphs())
@pytest.mark.parametrize("k", [3, 4, 5])
def test_dp_equals_brute_force(name, g, k):
    colors = gg.colors(g.n, k, seed=sum(map(ord, name)) + k)
    tab = O.Table(g, colors, k, O.ROOT_ALL)
    ref = brute.treelet_counts(g, colors, k)
    for h in range(1, k + 1):
        assert table_as_strings(tab, h) == ref[h], (name, k, h)


@pytest.mark.parametrize("k", [5, 6])
def test_dp_equals_pair_join(k):
    g = gg.erdos_renyi(12, 24, seed=3)
    colors = gg.colors(g.n, k, seed=9)
    tab = O.Table(g, colors, k, O.ROOT_ALL)
    ref = brute.pair_join_counts(g, colors, k)
    for h in range(1, k + 1):
        assert table_as_strings(tab, h) == ref[h]


def test_zero_rooting_keeps_colour_zero_roots():
    # Sec. 3.4: level k only at colour-0 vertices; lower levels unchanged
    g = gg.erdos_renyi(10, 20, seed=5)
    k = 4
    colors = gg.colors(g.n, k, seed=2)
    tz = O.Table(g, colors, k, O.ROOT_ZERO)
    ta = O.Table(g, colors, k, O.ROOT_ALL)
    for h in range(1, k):
        assert tz.level_dict(h) == ta.level_dict(h)
    full = ta.level_dict(k)
    assert tz.level_dict(k) == {key: c for key, c in full.items() if colors[key[0]] == 0}
    # P10: per unrooted shape, the all-rootings sum is k times the colour-0 sum;
    # both tables report the same number of copies
    assert tz.totals() == ta.totals()


# --------------------------------------------------------------------------
# P6, P7: colour-coding identities
# --------------------------------------------------------------------------

def test_exhaustive_colourings_identity():
    # sum over all k^n colourings of c(T_C, v) = h! k^(n-h) N(T, v), and
    # sum of t = k! k^(n-k) * (#k-subtrees)   (Sec. 2, p_k = k!/k^k)
    g = gg.erdos_renyi(7, 11, seed=11)
    n, k = g.n, 4
    km = key_map(k)
    acc = defaultdict(int)
    tsum = 0
    for cols in itertools.product(range(k), repeat=n):
        colors = np.array(cols, dtype=np.uint8)
        tab = O.Table(g, colors, k, O.ROOT_ALL)
        for h in range(1, k + 1):
            off, key, lo, hi = tab.export_level(h)
            for v in range(n):
                for q in range(off[v], off[v + 1]):
                    hh, r, mask = km[int(key[q])]
                    acc[(h, v, r, mask)] += int(lo[q]) | (int(hi[q]) << 64)
        tsum += tab.totals()[0]
    for h in range(1, k + 1):
        rc = brute.rooted_copies(g, h)
        for v in range(n):
            for r in range(O.num_shapes(h)):
                N = rc.get((v, O.shape_string(h, r)), 0)
                for mask in range(1 << k):
                    if bin(mask).count("1") == h:
                        assert acc.get((h, v, r, mask), 0) == math.factorial(h) * k ** (n - h) * N
    assert tsum == math.factorial(k) * k ** (n - k) * brute.count_subtrees(g, k)


def test_random_colourings_mean():
    # E[t] = p_k * (#k-subtrees); the mean over R colourings lies within 5
    # standard errors (the colouring concentration bounds of Sec. 2.3 set the scale)
    g = gg.erdos_renyi(24, 40, seed=4)
    k = 4
    N = brute.count_subtrees(g, k)
    pk = math.factorial(k) / k ** k
    ts = np.array([O.Table(g, gg.colors(g.n, k, seed=1000 + r), k).totals()[0] for r in range(400)], float)
    se = ts.std(ddof=1) / np.sqrt(len(ts))
    assert abs(ts.mean() - pk * N) < 5 * se


# --------------------------------------------------------------------------
# P8: closed forms
# --------------------------------------------------------------------------

def test_closed_forms_level2_and_stars():
    g = gg.chung_lu(300, 1500, 2.2, 60, seed=8)
    k = 5
    colors = gg.colors(g.n, k, seed=3)
    tab = O.Table(g, colors, k, O.ROOT_ALL)
    lev2 = table_as_strings(tab, 2)
    star = {h: O.shape_string(h, 0) for h in range(2, k + 1)}  # "1010..": star rooted at its centre
    levs = {h: table_as_strings(tab, h) for h in range(2, k + 1)}
    for v in range(g.n):
        nb = colors[g.neighbors(v)]
        Nj = np.bincount(nb, minlength=k)
        for j in range(k):
            if j == colors[v]:
                continue
            assert lev2.get((v, "10", (1 << j) | (1 << int(colors[v]))), 0) == Nj[j]
        # colourful h-star at its centre: product of per-colour neighbour counts
        for h in range(3, k + 1):
            others = [j for j in range(k) if j != colors[v]]
            for sub in itertools.combinations(others, h - 1):
                mask = (1 << int(colors[v])) | sum(1 << j for j in sub)
                expect = int(np.prod([int(Nj[j]) for j in sub]))
                assert levs[h].get((v, star[h], mask), 0) == expect


def test_closed_form_complete_graph():
    # in K_n with n_j vertices of colour j: c(T_C, v) = ((h-1)!/|Aut T|) prod_{j in C - c_v} n_j
    g = gg.complete(7)
    k = 5
    colors = np.array([0, 1, 1, 2, 3, 4, 4], dtype=np.uint8)
    nj = np.bincount(colors, minlength=k)
    tab = O.Table(g, colors, k, O.ROOT_ALL)
    for h in range(2, k + 1):
        lev = table_as_strings(tab, h)
        for v in range(g.n):
            cv = int(colors[v])
            for r in range(O.num_shapes(h)):
                s = O.shape_string(h, r)
                coef = math.factorial(h - 1) // brute.aut_rooted(s)
                for mask in range(1 << k):
                    if bin(mask).count("1") != h or not (mask >> cv & 1):
                        continue
                    prod = 1
                    for j in range(k):
                        if j != cv and mask >> j & 1:
                            prod *= int(nj[j])
                    assert lev.get((v, s, mask), 0) == coef * prod


def test_path_closed_form():
    # in a path every subtree is a subpath: c(path_h rooted at an end, C, v)
    # counts the colourful subpaths of h vertices starting at v
    g = gg.path(9)
    k = 4
    colors = np.array([0, 1, 2, 3, 0, 1, 2, 3, 0], dtype=np.uint8)
    tab = O.Table(g, colors, k, O.ROOT_ALL)
    lev = table_as_strings(tab, 4)
    end = "1" * 3 + "0" * 3
    for v in range(g.n):
        expect = 0
        for d in (1, -1):
            vs = [v + d * i for i in range(4)]
            if all(0 <= x < g.n for x in vs) and len({int(colors[x]) for x in vs}) == 4:
                expect += 1
        assert lev.get((v, end, 0b1111), 0) == expect


# --------------------------------------------------------------------------
# Errors
# --------------------------------------------------------------------------

def test_invalid_inputs_rejected():
    g = gg.path(4)
    with pytest.raises(O.OracleError):
        O.Table(g, np.array([0, 1, 2, 4], np.uint8), 4)       # colour >= k
    with pytest.raises(O.OracleError):
        O.Table(g, np.zeros(4, np.uint8), 9)                  # k > 8
    bad = gg.Graph(3, np.array([0, 1, 1, 1]), np.array([1], np.int32))  # asymmetric
    assert O.check_csr(bad) != 0
    loop = gg.Graph(2, np.array([0, 1, 1]), np.array([0], np.int32))
    assert O.check_csr(loop) != 0


def test_overflow_reported_not_wrapped():
    # Sec. 3.2 footnote: a 6-star at a hub of degree 2^16 has ~1e22 copies;
    # at k = 8 a hub of degree ~2e5 gives a colourful 8-star count near 2^103,
    # which 128-bit counts hold exactly. The oracle carries them without error.
    leaves = 1 << 16
    g = gg.star(leaves)
    k = 6
    colors = np.concatenate([[0], (np.arange(leaves) % 5) + 1]).astype(np.uint8)
    tab = O.Table(g, colors, k, O.ROOT_ZERO)
    per = np.bincount(colors[1:], minlength=k)[1:]
    expect = math.prod(int(x) for x in per)
    assert tab.totals()[0] == expect
    assert expect > 2 ** 64


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------

def test_philox_matches_numpy():
    # numpy's Philox (4x64, 10 rounds) increments its counter before each block
    for key, ctr in [((0, 0), (0, 0, 0, 0)), ((5, 7), (41, 3, 9, 1)), ((2**64 - 1, 12345), (2**64 - 1, 2**64 - 1, 0, 7))]:
        bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(ctr, np.uint64))
        ref = [int(x) for x in bg.random_raw(4)]
        nxt = list(ctr)
        for i in range(4):
            nxt[i] = (nxt[i] + 1) % 2**64
            if nxt[i] != 0:
                break
        assert O.philox4x64(nxt, key) == ref


def test_uniform_below_range_and_rejection():
    vals = [O.uniform_below(6, 1, 2, i, 0) for i in range(3000)]
    assert min(vals) == 0 and max(vals) == 5
    counts = np.bincount(vals, minlength=6)
    assert np.all(np.abs(counts - 500) < 5 * np.sqrt(500))
    big = 3 * 2**100 + 17
    assert all(O.uniform_below(big, 3, 4, i, 5) < big for i in range(200))
    assert O.uniform_below(1, 3, 4, 0, 0) == 0
