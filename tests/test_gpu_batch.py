"""Batched build (one persistent launch) vs the plain build, bit for bit.

Every instance of a batch must give the same table as scc_build_table on its
own: every level, totals, and the sample stream. Batches mix graph families,
sizes and k, force the chunked hub path and ragged vertex tiles, run the
autotuner, and route instances above a size to the level kernels.
"""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from gpu_util import assert_tables_equal, scc

pytestmark = pytest.mark.gpu


def instances(seed0=0):
    out = []
    specs = [("er", 300, 900, 2), ("cl", 2000, 8000, 5), ("ba", 500, 2, 6), ("er", 60, 150, 8),
             ("cl", 800, 3000, 7), ("lol", 9, 4, 4), ("er", 1, 0, 3), ("cl", 5000, 25000, 6),
             ("ba", 1200, 3, 5), ("star", 300, 0, 6)]
    for i, (kind, a, b, k) in enumerate(specs):
        if kind == "er":
            g = gg.erdos_renyi(a, b, seed=seed0 + i) if a > 1 else gg.csr_from_edges(1, np.zeros((0, 2), np.int64))
        elif kind == "cl":
            g = gg.chung_lu(a, b, 2.2, a / 20, seed=seed0 + i)
        elif kind == "ba":
            g = gg.barabasi_albert(a, b, seed=seed0 + i)
        elif kind == "star":
            g = gg.star(a)
        else:
            g = gg.lollipop(a, b)
        out.append((g, gg.colors(g.n, k, seed=seed0 + 50 + i), k))
    return out


def plain(S, g, colors, k, rooting):
    return S.Table(S.DeviceGraph.from_graph(g), colors, k, rooting=rooting)


@pytest.mark.parametrize("rooting", [0, 1])
@pytest.mark.parametrize("tile,hub,waves", [(0, 0, 0), (7, 16, 8), (1000, 40, 0), (64, 1024, 8)])
def test_batch_equals_plain(rooting, tile, hub, waves):
    S = scc()
    inst = instances()
    dev = [(S.DeviceGraph.from_graph(g), c, k) for g, c, k in inst]
    tabs, rep = S.build_batch(dev, rooting=rooting, tile=tile, hub_degree=hub, waves=waves)
    assert rep["waves"] == waves
    assert rep["items"] > 0 and rep["grid"] > 0
    for (g, c, k), bt in zip(inst, tabs):
        pt = plain(S, g, c, k, rooting)
        for h in range(1, k + 1):
            for x, y in zip(bt.export_level(h), pt.export_level(h)):
                assert np.array_equal(x, y), (g.n, k, h)
        assert bt.totals() == pt.totals()
        if pt.totals()[0]:
            a, pa = bt.sample(200, seed=3)
            b, pb = pt.sample(200, seed=3)
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
            assert np.array_equal(pa.cpu().numpy(), pb.cpu().numpy())


def test_batch_equals_oracle_and_autotune():
    S = scc()
    inst = instances(seed0=100)[:6]
    dev = [(S.DeviceGraph.from_graph(g), c, k) for g, c, k in inst]
    tabs, rep = S.build_batch(dev, autotune=True)
    assert rep["tuned"] and len(rep["probes"]) >= 2
    for (g, c, k), bt in zip(inst, tabs):
        assert_tables_equal(bt, O.Table(g, c, k, O.ROOT_ZERO), k, f"batch n={g.n} k={k}")
    # a second batch of the same shape reuses the tuned schedule
    tabs2, rep2 = S.build_batch(dev, autotune=True)
    assert rep2["tuned"] and not rep2["probes"]
    assert (rep2["tile"], rep2["hub_degree"]) == (rep["tile"], rep["hub_degree"])


def test_batch_with_wide_counts():
    S = scc()
    leaves = 1 << 16
    edges = [(0, i) for i in range(1, leaves + 1)] + [(i, i + 1) for i in range(1, 200)]
    g = gg.csr_from_edges(leaves + 1, np.array(edges, np.int64))
    colors = np.concatenate([[0], (np.arange(leaves) % 5) + 1]).astype(np.uint8)
    small = gg.erdos_renyi(100, 300, seed=1)
    dev = [(S.DeviceGraph.from_graph(g), colors, 6), (S.DeviceGraph.from_graph(small), gg.colors(100, 6, seed=2), 6)]
    tabs, _ = S.build_batch(dev)
    assert_tables_equal(tabs[0], O.Table(g, colors, 6), 6, "wide star in a batch")
    assert tabs[0].totals()[0] > 2 ** 64


@pytest.mark.parametrize("rooting", [0, 1])
def test_batch_with_128_bit_neighbour_sums(rooting):
    # a hub of 2^17 leaves at k = 7: the hub's level-6 counts exceed 2^64, so the
    # leaves' level-6 neighbour sums have nonzero high words, which the batched
    # worker stages beside the low words for the level-7 combine
    S = scc()
    leaves = 1 << 17
    edges = [(0, i) for i in range(1, leaves + 1)] + [(i, i + 1) for i in range(1, 200)]
    g = gg.csr_from_edges(leaves + 1, np.array(edges, np.int64))
    colors = np.concatenate([[0], (np.arange(leaves) % 6) + 1]).astype(np.uint8)
    small = gg.erdos_renyi(100, 300, seed=1)
    dev = [(S.DeviceGraph.from_graph(small), gg.colors(100, 7, seed=2), 7), (S.DeviceGraph.from_graph(g), colors, 7)]
    tabs, _ = S.build_batch(dev, rooting=rooting, tile=512, hub_degree=1024, waves=8)
    assert_tables_equal(tabs[1], O.Table(g, colors, 7, rooting), 7, "128-bit sums in a batch")
    assert tabs[1].occ(0, -1) > 2 ** 64


def test_batch_zero_rooting_colour_zero_sparse():
    # zero-rooting: the level-k combine and the level k-1 gather visit only the
    # colour-0 vertices of each tile (none, one, or about a k-th of them)
    S = scc()
    inst = []
    for i, k in enumerate([4, 6, 7]):
        g = gg.chung_lu(3000, 12000, 2.2, 300, seed=40 + i)
        c = (gg.colors(g.n, k - 1, seed=60 + i) + 1).astype(np.uint8)      # no colour 0
        inst.append((g, c, k))
        c1 = c.copy()
        c1[[5, 1500, 2999]] = 0                                               # three colour-0 vertices
        inst.append((g, c1, k))
        inst.append((g, gg.colors(g.n, k, seed=70 + i), k))                   # uniform colours
    dev = [(S.DeviceGraph.from_graph(g), c, k) for g, c, k in inst]
    tabs, _ = S.build_batch(dev, tile=100, hub_degree=64, waves=8)
    for (g, c, k), bt in zip(inst, tabs):
        assert_tables_equal(bt, O.Table(g, c, k, O.ROOT_ZERO), k, f"batch colour-0 n={g.n} k={k}")


@pytest.mark.parametrize("plain_nnz", [5000, 1, -1])
def test_batch_scheduler_routes_large_instances_to_the_level_kernels(plain_nnz):
    # instances with at least plain_nnz CSR entries are built by the level
    # kernels before the persistent launch; every table is the same either way
    S = scc()
    inst = instances(seed0=200)
    dev = [(S.DeviceGraph.from_graph(g), c, k) for g, c, k in inst]
    tabs, rep = S.build_batch(dev, plain_nnz=plain_nnz, tile=64, hub_degree=1024)
    want = sum(1 for g, _, _ in inst if plain_nnz > 0 and g.nnz >= plain_nnz)
    assert rep["plain_instances"] == want
    if want < len(inst):
        assert rep["items"] > 0
    for (g, c, k), bt in zip(inst, tabs):
        pt = plain(S, g, c, k, 0)
        for h in range(1, k + 1):
            for x, y in zip(bt.export_level(h), pt.export_level(h)):
                assert np.array_equal(x, y), (g.n, k, h)
        assert bt.totals() == pt.totals()
    for (g, c, k), bt in list(zip(inst, tabs))[:4]:
        assert_tables_equal(bt, O.Table(g, c, k, O.ROOT_ZERO), k, f"scheduled batch n={g.n} k={k}")


@pytest.mark.parametrize("bad", ["plain", "persistent"])
def test_batch_scheduler_error_in_either_half(bad):
    # one invalid instance (a colour >= k) on either side of the scheduler: the call
    # fails with EINVAL after the other side has finished, and returns no table
    S = scc()
    inst = instances(seed0=300)
    dev = [(S.DeviceGraph.from_graph(g), c.copy(), k) for g, c, k in inst]
    big = [i for i, (g, _, _) in enumerate(inst) if g.nnz >= 5000]
    small = [i for i, (g, _, _) in enumerate(inst) if 0 < g.nnz < 5000]
    assert big and small
    i = big[0] if bad == "plain" else small[0]
    g, c, k = dev[i]
    c[0] = k
    dev[i] = (g, c, k)
    with pytest.raises(S.SccError) as e:
        S.build_batch(dev, plain_nnz=5000)
    assert e.value.status == S.EINVAL
    # the library is still usable afterwards
    tabs, rep = S.build_batch([x for j, x in enumerate(dev) if j != i], plain_nnz=5000)
    assert rep["plain_instances"] == len(big) - (1 if bad == "plain" else 0)
