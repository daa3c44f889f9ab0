"""Pins of the sparse k <= 16 oracle (oracle/oracle16.c, Sec. 3.2 generality).

* k = 3..8: every level equals the table of the k <= 8 oracle (itself pinned by
  brute force, closed forms and the paper's fixtures), keys translated from
  (DFS bitstring, colour set) to the ITE numbering;
* k = 9 and 10: every level equals brute-force enumeration of colourful
  subtrees rooted at every vertex (the definition of c(T_C, v), Sec. 2.1), and
  t equals the number of colourful k-subtrees;
* k = 12 and 16: a star's counts at its centre are the products of the colour
  class sizes (closed form), and every level-h count of a path graph equals the
  brute-force count.
"""
from __future__ import annotations

from collections import Counter
from math import prod

import numpy as np
import pytest

import brute
import graphgen as gg
import oracle as O


def _ite_key(k, h, bits, mask, rank_of):
    return O.key(k, h, rank_of[h][bits], mask)


def _rank_maps(k):
    out = {}
    for h in range(1, k + 1):
        out[h] = {}
        for r in range(O.num_shapes(h)):
            s = O.shape_string(h, r)
            out[h][int(s, 2) if s else 0] = r
    return out


@pytest.mark.parametrize("k", [3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("rooting", [O.ROOT_ZERO, O.ROOT_ALL])
def test_equals_the_k8_oracle(k, rooting):
    ranks = _rank_maps(k)
    for g in (gg.erdos_renyi(40 if k <= 6 else 26, 90 if k <= 6 else 50, seed=10 + k),
              gg.chung_lu(60, 150, 2.2, 12, seed=20 + k), gg.lollipop(7, 3)):
        colors = gg.colors(g.n, k, seed=30 + k + rooting)
        a = O.Table(g, colors, k, rooting)
        b = O.Table16(g, colors, k, rooting)
        for h in range(1, k + 1):
            want = a.level_dict(h)
            got = {}
            for (v, key), c in b.level_dict(h).items():
                got[(v, _ite_key(k, h, key >> 16, key & 0xffff, ranks))] = c
            assert got == want, (k, h)
        assert b.total() == a.totals()[0]


def _brute16(g, colors, k):
    """{h: {(v, key16): count}} from brute-force subtree enumeration."""
    out = {}
    for h, d in brute.treelet_counts(g, colors, k).items():
        out[h] = {(v, O.key16(int(s, 2) if s else 0, mask)): c for (v, s, mask), c in d.items()}
    return out


@pytest.mark.parametrize("k,seed", [(9, 1), (10, 3)])
def test_equals_brute_force_at_k9_k10(k, seed):
    # a random tree on 13 vertices plus a few chords: many 9- and 10-vertex subtrees
    rng = np.random.default_rng(seed)
    n = 13
    edges = {(int(rng.integers(0, v)), v) for v in range(1, n)}
    while len(edges) < n + 3:
        a, b = sorted(int(x) for x in rng.choice(n, 2, replace=False))
        edges.add((a, b))
    g = gg.csr_from_edges(n, np.array(sorted(edges), np.int64))
    colors = (rng.permutation(n) % k).astype(np.uint8)        # every colour present
    want = _brute16(g, colors, k)
    tab = O.Table16(g, colors, k, O.ROOT_ALL)
    for h in range(1, k + 1):
        assert tab.level_dict(h) == want[h], h
    n_colourful = sum(1 for vs, es in brute.subtrees(g, k) if len({int(colors[v]) for v in vs}) == k)
    assert tab.total() == n_colourful
    assert n_colourful > 0


@pytest.mark.parametrize("k,leaves", [(12, 40), (16, 60)])
def test_star_closed_form(k, leaves):
    g = gg.star(leaves)
    rng = np.random.default_rng(k)
    colors = np.concatenate([[0], rng.integers(1, k, leaves)]).astype(np.uint8)
    nj = Counter(int(c) for c in colors[1:])
    tab = O.Table16(g, colors, k, O.ROOT_ALL)
    for h in range(2, k + 1):
        star_bits = int("10" * (h - 1), 2)
        got = {key & 0xffff: c for (v, key), c in tab.level_dict(h).items() if v == 0 and key >> 16 == star_bits}
        for mask, c in got.items():
            assert mask & 1
            assert c == prod(nj[j] for j in range(1, k) if mask >> j & 1), (h, mask)
        # every colour set of size h holding colour 0 and colours present in the leaves
        present = [j for j in range(1, k) if nj[j] > 0]
        from itertools import combinations
        assert len(got) == sum(1 for _ in combinations(present, h - 1))


def test_path_levels_at_k16():
    g = gg.path(20)
    colors = (np.arange(20) % 16).astype(np.uint8)
    want = _brute16(g, colors, 16)
    tab = O.Table16(g, colors, 16, O.ROOT_ALL)
    for h in range(1, 17):
        assert tab.level_dict(h) == want[h], h
    assert tab.total() == sum(1 for i in range(20 - 15) if len(set(colors[i:i + 16])) == 16)


def test_u256_arithmetic():
    # the oracle's 256-bit add, multiply and small division against Python's integers
    M = 1 << 256
    rng = np.random.default_rng(9)
    cases = [(0, 0, 1), (M - 1, 1, 7), (M - 1, M - 1, 3), (1 << 128, 1 << 127, 5), (1 << 192, 1 << 64, 15),
             ((1 << 255) + 12345, 2, 16), (2 ** 64 - 1, 2 ** 64 - 1, 2 ** 64 - 1)]
    for _ in range(300):
        bits = rng.integers(1, 257, 2)
        a = int(rng.integers(0, 2 ** 62)) << int(max(0, bits[0] - 62)) | int(rng.integers(0, 2 ** 62))
        b = int(rng.integers(0, 2 ** 62)) << int(max(0, bits[1] - 62)) | int(rng.integers(0, 2 ** 62))
        cases.append((a % M, b % M, int(rng.integers(1, 2 ** 63))))
    for a, b, d in cases:
        s, p, q, r, so, po = O.u256_ops(a, b, d)
        assert s == (a + b) % M and so == (a + b >= M)
        assert p == (a * b) % M and po == (a * b >= M)
        assert q == a // d and r == a % d
