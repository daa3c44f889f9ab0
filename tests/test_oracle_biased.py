"""Pins of the oracle's biased colouring (Sec. 3.5, "Biased coloring").

* The colour of v comes from Philox (pinned against numpy's Philox elsewhere):
  the generator's first output word for counter (v, 0, 1, 0) is checked
  against numpy's, and the colour frequencies against the law (chi-square).
* Exact expectation: on a small graph, summing c(T_C, v) over all k^n
  colourings weighted by their probability under the biased law gives
  p_{k,h}(C) * N(T, v), with N(T, v) the number of (uncoloured) copies of the
  rooted tree T at v from brute force and p_{k,h}(C) = h! lambda^h when colour
  0 is not in C, h! lambda^(h-1) (1 - (k-1) lambda) when it is; the paper
  prints only an approximation for the second case. Every level and key, in
  exact rational arithmetic.
"""
from __future__ import annotations

import itertools
from collections import defaultdict
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import graphgen as gg
import oracle as O
import brute


def _numpy_first_word(v, seed, stream):
    # numpy's Philox increments its counter before each block
    bg = np.random.Philox(key=np.array([seed, stream], np.uint64),
                          counter=np.array([(v - 1) % 2**64, 0 if v else 2**64 - 1, 1 if v else 0, 0], np.uint64))
    return int(bg.random_raw(1)[0])


def test_biased_colours_follow_philox():
    k, L, seed, stream = 6, O.lambda_units(0.05), 11, 3
    col = O.color_biased(300, k, L, seed, stream)
    t0 = 2**32 - (k - 1) * L
    for v in range(1, 300):
        r = _numpy_first_word(v, seed, stream) & 0xFFFFFFFF
        assert col[v] == (0 if r < t0 else 1 + (r - t0) // L), v


@pytest.mark.parametrize("k,lam", [(4, 0.05), (6, 0.01), (8, 0.1), (5, 0.2)])
def test_biased_colour_frequencies(k, lam):
    L = O.lambda_units(lam)
    n = 400_000
    col = O.color_biased(n, k, L, seed=7, stream=k)
    assert col.max() < k
    p = np.array([1 - (k - 1) * L / 2**32] + [L / 2**32] * (k - 1))
    obs = np.bincount(col, minlength=k)
    assert stats.chisquare(obs, p * n).pvalue > 1e-4


def test_biased_lambda_edges():
    # lambda = 1/(k-1) leaves colour 0 out entirely (k = 5: L = 2^30)
    edge = O.color_biased(4000, 5, 2**30, seed=1)
    assert (edge != 0).all() and set(edge.tolist()) == {1, 2, 3, 4}
    # the smallest lambda: almost every vertex gets colour 0
    tiny = O.color_biased(4000, 8, 1, seed=2)
    assert (tiny == 0).all()


def test_biased_lambda_out_of_range():
    with pytest.raises(O.OracleError):
        O.color_biased(10, 4, 0, seed=1)
    with pytest.raises(O.OracleError):
        O.color_biased(10, 4, 2**32 // 3 + 1, seed=1)


def _rooted_copies(g, h):
    """N(T, v): uncoloured copies of each rooted h-tree at each vertex, by brute force."""
    out = defaultdict(int)
    for vs, es in brute.subtrees(g, h):
        adj = defaultdict(set)
        for a, b in es:
            adj[a].add(b)
            adj[b].add(a)
        for r in vs:
            out[(r, brute.rooted_string(adj, r) if h > 1 else "")] += 1
    return out


def test_expected_counts_under_biased_law_exact():
    k = 4
    # a 5-vertex graph with a triangle, a pendant path and a chord
    g = gg.csr_from_edges(5, np.array([(0, 1), (1, 2), (0, 2), (2, 3), (3, 4), (1, 3)], np.int64))
    L = O.lambda_units(0.15)
    lam = Fraction(L, 2**32)
    pc = [1 - (k - 1) * lam] + [lam] * (k - 1)
    strings = {h: [O.shape_string(h, r) for r in range(O.num_shapes(h))] for h in range(1, k + 1)}
    decode = {}
    for h in range(1, k + 1):
        for r in range(O.num_shapes(h)):
            for C in range(1 << k):
                if bin(C).count("1") == h:
                    decode[O.key(k, h, r, C)] = (h, strings[h][r], C)
    got = defaultdict(Fraction)
    for cols in itertools.product(range(k), repeat=g.n):
        w = Fraction(1)
        for c in cols:
            w *= pc[c]
        tab = O.Table(g, np.array(cols, np.uint8), k, O.ROOT_ALL)
        for h in range(1, k + 1):
            off, key, lo, hi = tab.export_level(h)
            for v in range(g.n):
                for q in range(off[v], off[v + 1]):
                    got[(v,) + decode[int(key[q])]] += w * (int(lo[q]) | (int(hi[q]) << 64))
    expect = {}
    for h in range(1, k + 1):
        N = _rooted_copies(g, h)
        fact = 1
        for i in range(2, h + 1):
            fact *= i
        for (v, s), cnt in N.items():
            for C in range(1 << k):
                if bin(C).count("1") != h:
                    continue
                p = fact * (lam ** (h - 1) * (1 - (k - 1) * lam) if C & 1 else lam ** h)
                expect[(v, h, s if h > 1 else strings[1][0], C)] = p * cnt
                # the oracle's double-precision form of the same probability
                assert O.colour_set_prob(k, L, h, bool(C & 1)) == pytest.approx(float(p), rel=1e-12)
    assert {x: y for x, y in got.items() if y} == {x: y for x, y in expect.items() if y}
