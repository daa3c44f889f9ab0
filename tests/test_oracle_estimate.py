"""Pins of the oracle's estimators (Sec. 2.2) against what the paper and brute force fix.

* Ideal hits: a uniform colourful k-treelet copy spans class i with probability
  c_i sigma_i / t (Sec. 2.2), and t = sum_i c_i sigma_i. Feeding the hits a
  sampler would give in expectation (hits_i = c_i sigma_i out of n = t samples)
  must return c_i exactly, with c_i counted by brute force over the colourful
  induced k-subsets. A dropped sigma_i or t, or a swapped ratio, fails.
* Over every colouring of a small graph, the colourful copies of class i
  average to p_k times the copies of class i in G (p_k = k!/k^k): the mean of
  the graph-copy estimates c_i / p_k over all k^n colourings equals the
  brute-force count of induced copies of class i.
* AGS estimates are hits_i / w_i (Sec. 4.1), 0 where w_i = 0.
"""
from __future__ import annotations

import itertools
from collections import Counter

import numpy as np
import pytest

import brute
import graphgen as gg
import oracle as O


def _class_counts(g, colors, k):
    out = Counter()
    for vs, _ in brute.colourful_graphlets(g, colors, k):
        out[int(O.classify(g, k, np.array([vs], np.int32))[1][0])] += 1
    return out


def _sigma(k):
    return [O.spanning_trees(int(c), k) for c in O.catalog_codes(k)]


@pytest.mark.parametrize("k,seed", [(4, 1), (5, 2)])
def test_ideal_hits_give_the_colourful_counts(k, seed):
    g = gg.erdos_renyi(14, 30, seed=seed)
    colors = gg.colors(g.n, k, seed=10 + seed)
    tab = O.Table(g, colors, k)
    t, _ = tab.totals()
    truth = _class_counts(g, colors, k)
    sig = _sigma(k)
    hits = np.array([truth.get(i, 0) * sig[i] for i in range(len(sig))], np.int64)
    assert int(hits.sum()) == t                       # t = sum_i c_i sigma_i
    c, gest = O.estimate(tab, hits, n=t)
    for i in range(len(sig)):
        assert c[i] == pytest.approx(truth.get(i, 0), rel=1e-12, abs=1e-12), i
    pk = 1.0
    for i in range(1, k + 1):
        pk *= i / k
    assert np.allclose(gest, c / pk, rtol=1e-15, atol=0)


def test_graph_copy_estimates_average_to_the_graphlet_counts():
    k = 4
    g = gg.csr_from_edges(6, np.array([(0, 1), (1, 2), (2, 3), (3, 0), (0, 2), (3, 4), (4, 5), (2, 5)], np.int64))
    # induced copies of each class in G, by brute force over all 4-subsets
    allc = np.zeros(g.n, np.uint8)
    exact = Counter()
    for vs in itertools.combinations(range(g.n), k):
        sub = g.n and brute.connected_subsets  # noqa: F841 (documentation: connectivity checked below)
        adj = {v: set(int(u) for u in g.neighbors(v)) & set(vs) for v in vs}
        seen, stack = {vs[0]}, [vs[0]]
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if y not in seen:
                    seen.add(y)
                    stack.append(y)
        if len(seen) == k:
            exact[int(O.classify(g, k, np.array([vs], np.int32))[1][0])] += 1
    sig = _sigma(k)
    total = np.zeros(len(sig))
    ncol = 0
    for cols in itertools.product(range(k), repeat=g.n):
        colors = np.array(cols, np.uint8)
        ncol += 1
        truth = _class_counts(g, colors, k)
        if not truth:
            continue
        tab = O.Table(g, colors, k)
        t, _ = tab.totals()
        hits = np.array([truth.get(i, 0) * sig[i] for i in range(len(sig))], np.int64)
        _, gest = O.estimate(tab, hits, n=t)
        total += gest
    mean = total / ncol
    for i in range(len(sig)):
        assert mean[i] == pytest.approx(exact.get(i, 0), rel=1e-9, abs=1e-9), (i, mean[i], exact.get(i, 0))
    assert sum(exact.values()) > 0 and len(exact) >= 3


def test_ags_estimates_are_hits_over_weights():
    k = 4
    g = gg.lollipop(8, 3)
    tab = O.Table(g, gg.colors(g.n, k, seed=3), k)
    s = O.num_classes(k)
    hits = np.arange(s, dtype=np.int64) * 7
    w = np.linspace(0.0, 2.5, s)
    c, gest = O.estimate(tab, hits, w=w)
    for i in range(s):
        assert c[i] == (hits[i] / w[i] if w[i] > 0 else 0.0)
    with pytest.raises(O.OracleError):
        O.estimate(tab, hits, n=0)                    # uniform estimates need samples
