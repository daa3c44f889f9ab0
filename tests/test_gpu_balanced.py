"""Round skipping (Sec. 3.3, balanced decomposition) on the GPU vs the oracle, bit for bit.

* Tables built with the balanced rooting: every level (level k-1 empty, level
  k holding only the designated rootings, at every vertex), t, the
  orbit-divided t_j and the number of stars, for random graphs and every k in
  [4, 8], with and without the chunked hub gather.
* The non-star t_j equal those of the zero-rooting table built on the GPU, a
  property that holds at any size (checked on multi-tile graphs and on the
  mid-size workload, Chung-Lu n = 1e6, m = 1e7, k = 6).
* Samples: the shape-first uniform draw, every non-star shape and the direct
  star sampler equal the oracle's row by row; at the mid size they are valid
  trees (and stars) of the graph.
* Counts above 2^64 (a hub of 2^17 neighbours), degenerate inputs (k < 4, no
  non-star copy, no star), a server mixing the three kinds of request, and the
  batched build, AGS and AGS sessions refusing the mode.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from gpu_util import assert_tables_equal, build_pair, random_graphs, scc

pytestmark = pytest.mark.gpu

BAL = O.ROOT_BALANCED


def _assert_samples(gt, ot, n, seed, shape, stream=0, first=0, label=""):
    gv, gp = gt.sample(n, seed=seed, stream_id=stream, shape=shape, first_index=first)
    ov, op = ot.sample(n, seed=seed, stream=stream, shape=shape, first_index=first)
    assert np.array_equal(gv.cpu().numpy(), ov), f"{label} shape {shape}: vertices differ"
    assert np.array_equal(gp.cpu().numpy(), op), f"{label} shape {shape}: parents differ"


def test_designated_rootings_agree():
    S = scc()
    for k in range(2, 9):
        assert S.star_shape(k) == O.star_class(k)
        for j in range(S.num_unrooted(k)):
            assert S.balanced_rooting(k, j) == (O.balanced_rank(k, j), O.balanced_orbit(k, j)), (k, j)


@pytest.mark.parametrize("k", [4, 5, 6, 7, 8])
@pytest.mark.parametrize("hub_degree", [0, 6])
def test_balanced_tables_every_k(k, hub_degree):
    for name, g in random_graphs(k):
        colors = gg.colors(g.n, k, seed=23 * k + 1)
        gt, ot = build_pair(g, colors, k, rooting=BAL, hub_degree=hub_degree)
        assert_tables_equal(gt, ot, k, f"{name} balanced hub>{hub_degree}")
        assert gt.info().nnz[k - 1] == 0
        assert gt.star_count() == ot.star_count() == sum(math.comb(int(d), k - 1) for d in g.degrees())


@pytest.mark.parametrize("k", [4, 5, 6, 7, 8])
@pytest.mark.parametrize("hub_degree", [0, 6])
def test_balanced_samples_every_k(k, hub_degree):
    for name, g in random_graphs(k):
        colors = gg.colors(g.n, k, seed=23 * k + 1)
        gt, ot = build_pair(g, colors, k, rooting=BAL, hub_degree=hub_degree)
        t, tj = ot.totals()
        if t:
            _assert_samples(gt, ot, 1500, seed=7 + k, shape=-1, stream=3, first=11, label=name)
        for j in range(O.num_unrooted(k)):
            if j != O.star_class(k) and tj[j]:
                _assert_samples(gt, ot, 300, seed=100 + j, shape=j, stream=j, label=name)
        if ot.star_count():
            _assert_samples(gt, ot, 800, seed=5, shape=O.star_class(k), stream=9, first=1 << 33, label=name)


@pytest.mark.parametrize("k,n,m,wmax", [(6, 20000, 100000, 2000), (8, 3000, 12000, 300)])
def test_balanced_totals_equal_zero_rooting(k, n, m, wmax):
    S = scc()
    g = gg.chung_lu(n, m, 2.2, wmax, seed=31 + k)
    colors = gg.colors(g.n, k, seed=32)
    dg = S.DeviceGraph.from_graph(g)
    zt = S.Table(dg, colors, k, rooting=O.ROOT_ZERO)
    bt = S.Table(dg, colors, k, rooting=BAL)
    t0, tj0 = zt.totals()
    t1, tj1 = bt.totals()
    star = O.star_class(k)
    assert tj1 == [0 if j == star else tj0[j] for j in range(len(tj0))]
    assert t1 == t0 - tj0[star]
    assert bt.star_count() == sum(math.comb(int(d), k - 1) for d in g.degrees())
    # levels below k-1 do not depend on the rooting
    for h in range(1, k - 1):
        for a, b in zip(zt.export_level(h), bt.export_level(h)):
            assert np.array_equal(a, b), h


def test_balanced_wide_counts():
    # a hub of 2^17 leaves (six leaf colours) with a path through 200 of them: at
    # k = 7 the hub's stars (about 7e27) and a designated count at the hub exceed
    # 2^64, and the hub's per-vertex bound sends it through the 128-bit combine
    leaves = 1 << 17
    edges = [(0, i) for i in range(1, leaves + 1)] + [(i, i + 1) for i in range(1, 200)]
    g = gg.csr_from_edges(leaves + 1, np.array(edges, np.int64))
    colors = np.concatenate([[0], (np.arange(leaves) % 6) + 1]).astype(np.uint8)
    gt, ot = build_pair(g, colors, 7, rooting=BAL)
    assert_tables_equal(gt, ot, 7, "wide balanced")
    assert gt.star_count() == ot.star_count() > 2 ** 64
    assert max(gt.totals()[1]) > 2 ** 64
    assert gt.info().wide_vertices[7] >= 1
    _assert_samples(gt, ot, 2000, seed=3, shape=-1, label="wide")
    _assert_samples(gt, ot, 2000, seed=4, shape=O.star_class(7), label="wide")


def test_balanced_degenerate_and_refusals():
    S = scc()
    # k < 4 has no balanced decomposition
    g = gg.erdos_renyi(30, 60, seed=1)
    with pytest.raises(S.SccError) as e:
        S.Table(S.DeviceGraph.from_graph(g), gg.colors(g.n, 3, seed=1), 3, rooting=BAL)
    assert e.value.status == S.EINVAL
    # a star graph: every 4-treelet is a star, so t = 0 but the stars are sampled
    star = gg.csr_from_edges(6, np.array([(0, i) for i in range(1, 6)], np.int64))
    colors = np.array([0, 1, 2, 3, 1, 2], np.uint8)
    gt, ot = build_pair(star, colors, 4, rooting=BAL)
    assert_tables_equal(gt, ot, 4, "star graph")
    assert gt.totals()[0] == 0 and gt.star_count() == 10
    with pytest.raises(S.SccError) as e:
        gt.sample(5, seed=1)
    assert e.value.status == S.EEMPTY
    _assert_samples(gt, ot, 200, seed=2, shape=O.star_class(4), label="star graph")
    # a path: no 5-star, and every shape the path holds is sampled
    path = gg.csr_from_edges(40, np.array([(i, i + 1) for i in range(39)], np.int64))
    colors = gg.colors(40, 5, seed=3)
    gt, ot = build_pair(path, colors, 5, rooting=BAL)
    assert_tables_equal(gt, ot, 5, "path")
    assert gt.star_count() == 0
    with pytest.raises(S.SccError) as e:
        gt.sample(5, seed=1, shape=O.star_class(5))
    assert e.value.status == S.EEMPTY
    if gt.totals()[0]:
        _assert_samples(gt, ot, 200, seed=4, shape=-1, label="path")
    # AGS, AGS sessions and the batched build refuse the mode
    g = gg.erdos_renyi(200, 800, seed=5)
    colors = gg.colors(g.n, 5, seed=6)
    dg = S.DeviceGraph.from_graph(g)
    bt = S.Table(dg, colors, 5, rooting=BAL)
    with pytest.raises(S.SccError) as e:
        bt.ags(cbar=10, round_size=10, budget=100, seed=1)
    assert e.value.status == S.EINVAL
    srv = S.Server([bt], hbm_budget=8 << 20)
    with pytest.raises(S.SccError) as e:
        srv.ags_open(0, cbar=10, seed=1)
    assert e.value.status == S.EINVAL
    srv.close()
    with pytest.raises(S.SccError) as e:
        S.build_batch([(dg, colors, 5)], rooting=BAL)
    assert e.value.status == S.EINVAL


def test_balanced_server_mix_equals_alone():
    S = scc()
    g = gg.chung_lu(3000, 12000, 2.2, 150, seed=61)
    k = 6
    colors = gg.colors(g.n, k, seed=62)
    bt = S.Table(S.DeviceGraph.from_graph(g), colors, k, rooting=BAL)
    _, tj = bt.totals()
    shapes = [-1, O.star_class(k)] + [j for j, x in enumerate(tj) if x > 0][:4]
    rng = np.random.default_rng(63)
    reqs = [dict(table=0, n=int(rng.integers(10, 5000)), seed=int(rng.integers(1, 1 << 40)), stream_id=i,
                 first_index=int(rng.integers(0, 1 << 20)), shape=shapes[i % len(shapes)], classify=bool(i % 2))
            for i in range(18)]
    srv = S.Server([bt], hbm_budget=32 << 20, step_samples=2048, chunk=128)
    ids = [srv.submit(**q) for q in reqs]
    for q, rid in zip(reqs, ids):
        r = srv.wait(rid)
        assert r["status"] == 0
        v, p = bt.sample(q["n"], seed=q["seed"], stream_id=q["stream_id"], shape=q["shape"],
                         first_index=q["first_index"])
        assert np.array_equal(r["verts"].cpu().numpy(), v.cpu().numpy()), q
        assert np.array_equal(r["parent"].cpu().numpy(), p.cpu().numpy()), q
        if q["classify"]:
            assert np.array_equal(r["cls"].cpu().numpy(), bt.classify(v)[1].cpu().numpy()), q
        srv.release(rid)
    srv.close()
    ov, op = O.Table(g, colors, k, BAL).sample(reqs[0]["n"], seed=reqs[0]["seed"], stream=reqs[0]["stream_id"],
                                              shape=-1, first_index=reqs[0]["first_index"])
    v, p = bt.sample(reqs[0]["n"], seed=reqs[0]["seed"], stream_id=reqs[0]["stream_id"], shape=-1,
                     first_index=reqs[0]["first_index"])
    assert np.array_equal(v.cpu().numpy(), ov) and np.array_equal(p.cpu().numpy(), op)


def _has_edges(g, a, b):
    """vectorised edge test for arrays of endpoints"""
    lo, hi = g.row_ptr[a], g.row_ptr[a + 1]
    ok = np.zeros(len(a), bool)
    for i in range(len(a)):
        j = lo[i] + np.searchsorted(g.col_idx[lo[i]:hi[i]], b[i])
        ok[i] = j < hi[i] and g.col_idx[j] == b[i]
    return ok


@pytest.mark.timeout(600)
def test_balanced_mid_workload_properties():
    import torch
    S = scc()
    k = 6
    g = gg.chung_lu(1_000_000, 10_000_000, 2.1, 5e4, seed=2)
    colors = gg.colors(g.n, k, seed=3)
    dg = S.DeviceGraph.from_graph(g)
    zt = S.Table(dg, colors, k, rooting=O.ROOT_ZERO)
    bt = S.Table(dg, colors, k, rooting=BAL)
    zi, bi = zt.info(), bt.info()
    print(f"mid: zero-rooting {sum(zi.level_ms):.1f} ms {zi.bytes / 1e9:.2f} GB, "
          f"round skipping {sum(bi.level_ms):.1f} ms {bi.bytes / 1e9:.2f} GB", flush=True)
    t0, tj0 = zt.totals()
    t1, tj1 = bt.totals()
    star = O.star_class(k)
    assert tj1 == [0 if j == star else tj0[j] for j in range(len(tj0))]
    assert bt.star_count() == sum(math.comb(int(d), k - 1) for d in g.degrees())
    n = 4000
    for shape in (-1, star, int(np.argmax(tj1))):
        v, p = bt.sample(n, seed=17, shape=shape)
        torch.cuda.synchronize()
        sv, sp = v.cpu().numpy(), p.cpu().numpy()
        assert (sp[:, 0] == -1).all()
        assert all(len(set(row)) == k for row in sv.tolist())
        for q in range(1, k):
            assert ((sp[:, q] >= 0) & (sp[:, q] < q)).all()
            par = sv[np.arange(n), sp[:, q]]
            assert _has_edges(g, sv[:, q], par).all(), (shape, q)
        if shape == star:
            assert (sp[:, 1:] == 0).all()
        else:
            assert (np.sort(colors[sv], axis=1) == np.arange(k)).all()
