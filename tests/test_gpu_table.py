"""GPU table build vs the oracle, bit for bit (every level, every key, both count words).

Cases: the tiny workload (ER n=2000, m=8000, k=4, all rootings), random ER /
Chung-Lu / BA / lollipop graphs for every k in [2, 8] under both rootings,
multi-tile Chung-Lu graphs at k=6 and k=8, counts beyond 64 bits (a star with a
2^16-degree hub, the example in the paper's footnote on 128-bit counts), the
degenerate graphs (one vertex, isolated vertices, no colourful treelet), error
paths, and the full mid-size workload (Chung-Lu n=1e6, m=1e7, k=6).
"""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from gpu_util import assert_tables_equal, build_pair, random_graphs, scc

pytestmark = pytest.mark.gpu


def test_tiny_workload_all_rootings():
    g = gg.erdos_renyi(2000, 8000, seed=1)
    colors = gg.colors(g.n, 4, seed=11)
    gt, ot = build_pair(g, colors, 4, rooting=O.ROOT_ALL)
    assert_tables_equal(gt, ot, 4, "tiny")


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("rooting", [O.ROOT_ZERO, O.ROOT_ALL])
@pytest.mark.parametrize("hub_degree", [0, 6])
def test_random_graphs_every_k(k, rooting, hub_degree):
    # hub_degree = 6 sends every row of degree > 6 through the chunked hub gather
    for name, g in random_graphs(k):
        colors = gg.colors(g.n, k, seed=17 * k + rooting)
        gt, ot = build_pair(g, colors, k, rooting=rooting, hub_degree=hub_degree)
        assert_tables_equal(gt, ot, k, f"{name} hub>{hub_degree}")


@pytest.mark.parametrize("k", [3, 5, 7, 8])
@pytest.mark.parametrize("gather_mode", [1, 2])
def test_random_graphs_both_gather_modes(k, gather_mode):
    # grouped low-degree rows (1) and one row per wave (2), hub rows forced too
    for name, g in random_graphs(k):
        colors = gg.colors(g.n, k, seed=19 * k + gather_mode)
        for hub_degree in (0, 12):
            gt, ot = build_pair(g, colors, k, hub_degree=hub_degree, gather_mode=gather_mode)
            assert_tables_equal(gt, ot, k, f"{name} gather mode {gather_mode} hub>{hub_degree}")


@pytest.mark.parametrize("hub_degree", [0, 40])
@pytest.mark.parametrize("gather_mode", [0, 1, 2])
def test_chung_lu_k6_multi_tile(hub_degree, gather_mode):
    g = gg.chung_lu(20000, 100000, 2.1, 2000, seed=9)
    colors = gg.colors(g.n, 6, seed=10)
    gt, ot = build_pair(g, colors, 6, hub_degree=hub_degree, gather_mode=gather_mode)
    assert_tables_equal(gt, ot, 6, "cl20k")


@pytest.mark.parametrize("gather_mode", [1, 2])
def test_chung_lu_k8(gather_mode):
    g = gg.chung_lu(3000, 12000, 2.3, 300, seed=13)
    colors = gg.colors(g.n, 8, seed=14)
    gt, ot = build_pair(g, colors, 8, gather_mode=gather_mode)
    assert_tables_equal(gt, ot, 8, "cl3k-k8")


@pytest.mark.parametrize("gather_mode", [1, 2])
def test_counts_beyond_64_bits(gather_mode):
    # a 6-star at a hub of degree 2^16 has about 1e22 copies (Sec. 3.2 footnote);
    # the leaves' neighbour sums need 128 bits (grouped rows redo them alone)
    leaves = 1 << 16
    edges = [(0, i) for i in range(1, leaves + 1)] + [(i, i + 1) for i in range(1, 200)]
    g = gg.csr_from_edges(leaves + 1, np.array(edges, np.int64))
    colors = np.concatenate([[0], (np.arange(leaves) % 5) + 1]).astype(np.uint8)
    gt, ot = build_pair(g, colors, 6, gather_mode=gather_mode)
    assert_tables_equal(gt, ot, 6, "wide star")
    t, _ = gt.totals()
    assert t > 2 ** 64
    assert gt.info().wide_vertices[6] >= 1
    # with 64-bit counts only, the build refuses instead of wrapping
    S = scc()
    with pytest.raises(S.SccError) as e:
        S.Table(S.DeviceGraph.from_graph(g), colors, 6, max_bits=64)
    assert e.value.status == S.EOVERFLOW


@pytest.mark.parametrize("gather_mode", [1, 2])
def test_low_degree_rows_with_128_bit_sums(gather_mode):
    # a hub of 2^17 leaves at k = 7, all rootings: the hub's level-6 sum exceeds
    # 2^64, so the leaves (rows of one or two neighbours, grouped in mode 1) need
    # 128-bit neighbour sums at level 6 and are redone alone
    leaves = 1 << 17
    edges = [(0, i) for i in range(1, leaves + 1)] + [(i, i + 1) for i in range(1, 200)]
    g = gg.csr_from_edges(leaves + 1, np.array(edges, np.int64))
    colors = np.concatenate([[0], (np.arange(leaves) % 6) + 1]).astype(np.uint8)
    gt, ot = build_pair(g, colors, 7, rooting=O.ROOT_ALL, gather_mode=gather_mode)
    assert_tables_equal(gt, ot, 7, "hub k7")
    assert gt.occ(0, -1) > 2 ** 64


def test_degenerate_graphs():
    S = scc()
    # one vertex, no edges
    g1 = gg.csr_from_edges(1, np.zeros((0, 2), np.int64))
    gt, ot = build_pair(g1, np.zeros(1, np.uint8), 3)
    assert_tables_equal(gt, ot, 3, "single vertex")
    assert gt.totals()[0] == 0
    with pytest.raises(S.SccError) as e:
        gt.sample(4, seed=1)
    assert e.value.status == S.EEMPTY
    # isolated vertices mixed with a small component
    g2 = gg.csr_from_edges(30, np.array([(3, 4), (4, 5), (5, 6), (6, 3), (6, 20)], np.int64))
    colors = gg.colors(30, 4, seed=3)
    gt, ot = build_pair(g2, colors, 4, rooting=O.ROOT_ALL)
    assert_tables_equal(gt, ot, 4, "isolated")
    # a single colour: nothing colourful beyond level 1
    g3 = gg.erdos_renyi(50, 120, seed=5)
    gt, ot = build_pair(g3, np.zeros(50, np.uint8), 4)
    assert_tables_equal(gt, ot, 4, "monochrome")
    assert gt.totals()[0] == 0


@pytest.mark.parametrize("k", [3, 6])
def test_no_colour_zero_vertex(k):
    # zero-rooting with no vertex of colour 0: level k and its colour-0 row lists
    # are empty (no launch over them), every lower level is still stored
    g = gg.chung_lu(3000, 15000, 2.2, 300, seed=31)
    colors = (gg.colors(g.n, k - 1, seed=32) + 1).astype(np.uint8)
    gt, ot = build_pair(g, colors, k)
    assert_tables_equal(gt, ot, k, "no colour 0")
    assert gt.totals()[0] == 0
    # a single colour-0 vertex: level k holds its records only
    colors[17] = 0
    gt, ot = build_pair(g, colors, k)
    assert_tables_equal(gt, ot, k, "one colour-0 vertex")
    assert gt.info().nnz[k] == ot.level_nnz(k)


def test_invalid_inputs():
    S = scc()
    g = gg.erdos_renyi(20, 40, seed=1)
    dg = S.DeviceGraph.from_graph(g)
    with pytest.raises(S.SccError) as e:
        S.Table(dg, np.zeros(20, np.uint8), 9)
    assert e.value.status == S.EINVAL
    with pytest.raises(S.SccError) as e:
        S.Table(dg, gg.colors(20, 4, seed=2), 4, gather_mode=3)
    assert e.value.status == S.EINVAL
    bad_colors = gg.colors(20, 4, seed=2)
    bad_colors[3] = 4
    with pytest.raises(S.SccError) as e:
        S.Table(dg, bad_colors, 4, validate=True)
    assert e.value.status == S.EINVAL
    # asymmetric CSR: drop one direction of an edge
    rp, ci = g.row_ptr.copy(), g.col_idx.copy()
    v = int(np.argmax(np.diff(rp) > 0))
    ci2 = np.delete(ci, rp[v])
    rp2 = rp.copy()
    rp2[v + 1:] -= 1
    bad = S.DeviceGraph(rp2, ci2)
    with pytest.raises(S.SccError) as e:
        S.Table(bad, gg.colors(20, 4, seed=2), 4, validate=True)
    assert e.value.status == S.EINVAL


def test_occ_queries_match():
    g = gg.chung_lu(2000, 8000, 2.2, 200, seed=21)
    k = 6
    colors = gg.colors(g.n, k, seed=22)
    gt, ot = build_pair(g, colors, k)
    rng = np.random.default_rng(0)
    nk = O.num_keys(k)
    for _ in range(300):
        v = int(rng.integers(0, g.n))
        key = int(rng.integers(-1, nk))
        assert gt.occ(v, key) == ot.occ(v, key), (v, key)


@pytest.mark.timeout(900)
def test_mid_workload_full_table():
    # Chung-Lu n=1e6, m=1e7, exponent 2.1, k=6, zero-rooting: the whole table,
    # every level, bit for bit, then 300 samples of the bench's stream
    g = gg.chung_lu(1_000_000, 10_000_000, 2.1, 5e4, seed=2)
    colors = gg.colors(g.n, 6, seed=12)
    print("mid: graph ready", flush=True)
    gt, ot = build_pair(g, colors, 6, validate=False)
    print("mid: both tables built", flush=True)
    assert_tables_equal(gt, ot, 6, "mid")
    from gpu_util import assert_samples_equal
    assert_samples_equal(gt, ot, 300, seed=22, label="mid samples")
