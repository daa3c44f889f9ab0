"""The large workload (Chung-Lu n = 4e6, m = 6e7, exponent 2.3, w_max = 2e5, k = 8,
zero-rooting) at full size, checked by properties that hold at any size.

The oracle's full DP does not finish at this size, so the full table is pinned by
closed forms, and the smaller k = 8 graphs of the other tests carry the
entry-by-entry parity:
* a star rooted at its centre v with colour set C has exactly
  prod_{j in C, j != c_v} n_j(v) colourful copies, n_j(v) = number of neighbours
  of colour j (one distinct neighbour per leaf colour); checked through scc_occ
  at every level for the highest-degree vertices (whose counts need 128 bits)
  and for random ones;
* the total of the unrooted k-star is sum_v prod_{j != c_v} n_j(v) (each
  colourful star is rooted once, at its centre), exact over all 4e6 vertices;
* 10^4 samples are colourful trees of G (parents earlier in the row, every
  tree edge an edge of G, k distinct colours), and their induced-graphlet
  classes equal the oracle's classification of the same vertex sets.
"""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from gpu_util import scc

pytestmark = pytest.mark.gpu


def _has_edge(g, a, b):
    lo, hi = g.row_ptr[a], g.row_ptr[a + 1]
    i = lo + np.searchsorted(g.col_idx[lo:hi], b)
    return i < hi and g.col_idx[i] == b


@pytest.mark.timeout(900)
def test_large_k8_closed_forms_and_samples():
    S = scc()
    k = 8
    g = gg.chung_lu(4_000_000, 60_000_000, 2.3, 2e5, seed=3)
    colors = gg.colors(g.n, k, seed=13)
    print(f"large: n={g.n} m={g.m} d_max={int(g.degrees().max())}", flush=True)
    tab = S.Table(S.DeviceGraph.from_graph(g), colors, k, validate=False)
    info = tab.info()
    print(f"large: table {info.bytes / 1e9:.1f} GB, 128-bit vertices per level {list(info.wide_vertices)}", flush=True)
    assert sum(info.wide_vertices) > 0          # the hubs need 128 bits
    deg = np.diff(g.row_ptr)
    rows = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    nc = np.bincount(rows * k + colors[g.col_idx].astype(np.int64), minlength=g.n * k).reshape(g.n, k)
    del rows
    star = {h: next(r for r in range(O.num_shapes(h)) if O.shape_string(h, r) == "10" * (h - 1))
            for h in range(2, k + 1)}
    # the k-star total over every vertex
    prod = np.ones(g.n, dtype=object)
    for j in range(k):
        col = nc[:, j].astype(object)
        col[colors == j] = 1
        prod *= col
    expect = int(sum(prod))
    t, tj = tab.totals()
    assert tj[O.shape_unrooted(k, star[k])] == expect
    print(f"large: star total {expect} (t = {t})", flush=True)
    # rooted stars at every level: hubs and random vertices
    rng = np.random.default_rng(1)
    vs = np.concatenate([np.argsort(deg)[-24:], rng.choice(g.n, 200, replace=False)])
    checked = wide = 0
    for v in vs:
        v = int(v)
        cv = int(colors[v])
        others = [j for j in range(k) if j != cv]
        for h in range(2, k + 1):
            if h == k and cv != 0:
                continue                                 # level k is kept at colour-0 vertices only
            for _ in range(3):
                leaves = rng.choice(others, h - 1, replace=False)
                mask = (1 << cv) | sum(1 << int(j) for j in leaves)
                e = 1
                for j in leaves:
                    e *= int(nc[v, j])
                got = tab.occ(v, O.key(k, h, star[h], mask))
                assert got == e, (v, h, mask)
                checked += 1
                wide += e >= 1 << 64
    print(f"large: {checked} rooted-star counts checked, {wide} of them above 2^64", flush=True)
    assert wide > 0
    # samples: colourful trees of G, classified as the oracle classifies them
    n = 10_000
    vt, pt = tab.sample(n, seed=23)
    sv, sp = vt.cpu().numpy(), pt.cpu().numpy()
    assert (sp[:, 0] == -1).all()
    assert (np.sort(colors[sv], axis=1) == np.arange(k)).all()
    for i in range(n):
        for q in range(1, k):
            par = int(sp[i, q])
            assert 0 <= par < q
            assert _has_edge(g, int(sv[i, q]), int(sv[i, par])), (i, q)
    code, cls = tab.classify(vt)
    ocode, ocls = O.classify(g, k, sv)
    assert np.array_equal(code.cpu().numpy().view(np.uint32), ocode)
    assert np.array_equal(cls.cpu().numpy(), ocls)
