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
import torch
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


# (gather mode, width test): both gathers with the automatic width test, and
# each width test forced (one vertex per lane before the combine; inside it)
GATHER_WIDTH = [(1, 0), (2, 0), (0, 1), (0, 2)]


@pytest.mark.parametrize("gather_mode,width_test", GATHER_WIDTH)
def test_chung_lu_k8(gather_mode, width_test):
    g = gg.chung_lu(3000, 12000, 2.3, 300, seed=13)
    colors = gg.colors(g.n, 8, seed=14)
    gt, ot = build_pair(g, colors, 8, gather_mode=gather_mode, width_test=width_test)
    assert_tables_equal(gt, ot, 8, "cl3k-k8")


@pytest.mark.parametrize("gather_mode,width_test", GATHER_WIDTH)
def test_counts_beyond_64_bits(gather_mode, width_test):
    # a 6-star at a hub of degree 2^16 has about 1e22 copies (Sec. 3.2 footnote);
    # the leaves' neighbour sums need 128 bits (grouped rows redo them alone)
    leaves = 1 << 16
    edges = [(0, i) for i in range(1, leaves + 1)] + [(i, i + 1) for i in range(1, 200)]
    g = gg.csr_from_edges(leaves + 1, np.array(edges, np.int64))
    colors = np.concatenate([[0], (np.arange(leaves) % 5) + 1]).astype(np.uint8)
    gt, ot = build_pair(g, colors, 6, gather_mode=gather_mode, width_test=width_test)
    assert_tables_equal(gt, ot, 6, "wide star")
    t, _ = gt.totals()
    assert t > 2 ** 64
    info = gt.info()
    assert info.wide_vertices[6] >= 1
    # levels 4-6 have at most 64 outputs per vertex: four vertices per wave, the
    # hub (128-bit level-6 counts) passed on to the per-vertex combine (level 6
    # takes the width test per lane instead unless the test is forced per wave)
    if width_test != 1:
        assert info.grouped_combine >> 4 & 1 and info.grouped_combine >> 5 & 1, info.grouped_combine
    if width_test == 2:
        assert info.grouped_combine >> 6 & 1, info.grouped_combine
    # with 64-bit counts only, the build refuses instead of wrapping
    S = scc()
    with pytest.raises(S.SccError) as e:
        S.Table(S.DeviceGraph.from_graph(g), colors, 6, max_bits=64)
    assert e.value.status == S.EOVERFLOW


@pytest.mark.parametrize("gather_mode,width_test", GATHER_WIDTH)
def test_low_degree_rows_with_128_bit_sums(gather_mode, width_test):
    # a hub of 2^17 leaves at k = 7, all rootings: the hub's level-6 sum exceeds
    # 2^64, so the leaves (rows of one or two neighbours, grouped in mode 1) need
    # 128-bit neighbour sums at level 6 and are redone alone
    leaves = 1 << 17
    edges = [(0, i) for i in range(1, leaves + 1)] + [(i, i + 1) for i in range(1, 200)]
    g = gg.csr_from_edges(leaves + 1, np.array(edges, np.int64))
    colors = np.concatenate([[0], (np.arange(leaves) % 6) + 1]).astype(np.uint8)
    gt, ot = build_pair(g, colors, 7, rooting=O.ROOT_ALL, gather_mode=gather_mode, width_test=width_test)
    assert_tables_equal(gt, ot, 7, "hub k7")
    info = gt.info()
    if gather_mode == 2:
        # the hub's level-6 sum needs 128 bits: the rows are sorted before the gather
        assert info.sorted_sum_rows >> 6 & 1, info.sorted_sum_rows
    if width_test == 1:
        assert info.lane_width_test == sum(1 << h for h in range(4, 8))
    if width_test == 2:
        assert info.lane_width_test == 0
    # the leaves' level-6 sums are 128-bit, their own records are not
    assert sum(info.wide_input_rows[7][r] for r in (0, 1)) > 0
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
    for w in (-1, 3):
        with pytest.raises(S.SccError) as e:
            S.Table(dg, gg.colors(20, 4, seed=2), 4, width_test=w)
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


def test_invalid_inputs_rejected_by_default():
    # validation is the default (no flag): malformed CSRs and colours give EINVAL
    # before any kernel reads col_idx through them; rows whose bounds leave
    # [0, nnz] are caught by the first pass, which reads row_ptr only
    S = scc()
    g = gg.erdos_renyi(30, 60, seed=3)
    colors = gg.colors(30, 5, seed=4)
    cases = {}
    c = colors.copy(); c[7] = 5
    cases["colour >= k"] = (g.row_ptr, g.col_idx, c)
    rp = g.row_ptr.copy(); rp[10] = rp[-1] + 1000          # row bounds past nnz
    cases["row_ptr past nnz"] = (rp, g.col_idx, colors)
    rp = g.row_ptr.copy(); rp[5] = -3
    cases["negative row_ptr"] = (rp, g.col_idx, colors)
    rp = g.row_ptr.copy(); rp[0] = 1
    cases["row_ptr[0] != 0"] = (rp, g.col_idx, colors)
    rp = g.row_ptr.copy(); rp[-1] -= 1
    cases["row_ptr[n] != nnz"] = (rp, g.col_idx, colors)
    ci = g.col_idx.copy(); ci[3] = 30
    cases["neighbour out of range"] = (g.row_ptr, ci, colors)
    ci = g.col_idx.copy(); v = 2; ci[g.row_ptr[v]] = v
    cases["self-loop"] = (g.row_ptr, ci, colors)
    v = int(np.argmax(np.diff(g.row_ptr) >= 2))
    ci = g.col_idx.copy(); a = g.row_ptr[v]; ci[a], ci[a + 1] = ci[a + 1], ci[a]
    cases["unsorted row"] = (g.row_ptr, ci, colors)
    for name, (rp, ci, col) in cases.items():
        print("invalid case:", name, flush=True)
        with pytest.raises(S.SccError) as e:
            S.Table(S.DeviceGraph(rp, ci), col, 5)
        assert e.value.status == S.EINVAL, name
        # the host-graph form is checked the same way
        host = type("HostGraph", (), {"row_ptr": rp, "col_idx": ci})()
        with pytest.raises(S.SccError) as e:
            S.Table(host, col, 5)
        assert e.value.status == S.EINVAL, name
    # an empty graph is valid
    empty = S.Table(S.DeviceGraph(np.zeros(1, np.int64), np.zeros(0, np.int32)), np.zeros(0, np.uint8), 4)
    assert empty.totals()[0] == 0


def test_host_graph_equals_device_graph():
    # on_device = 0: the library copies the host CSR and colours; the table is
    # the device-graph table and the oracle's, bit for bit, and sampling and
    # classification read the table's own copies
    S = scc()
    g = gg.chung_lu(3000, 12000, 2.2, 150, seed=41)
    k = 6
    colors = gg.colors(g.n, k, seed=42)
    host = S.Table(g, colors.copy(), k)
    dev, ot = build_pair(g, colors, k)
    assert_tables_equal(host, ot, k, "host graph")
    hv, hp = host.sample(500, seed=5)
    dv, dp = dev.sample(500, seed=5)
    assert torch.equal(hv, dv) and torch.equal(hp, dp)
    assert torch.equal(host.classify(hv)[1], dev.classify(dv)[1])


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
    assert all(gt.info().grouped_combine >> h & 1 for h in (4, 5, 6))
    assert_tables_equal(gt, ot, 6, "mid")
    from gpu_util import assert_samples_equal
    assert_samples_equal(gt, ot, 300, seed=22, label="mid samples")


@pytest.mark.timeout(900)
def test_k8_counts_beyond_64_bits():
    # k = 8 with 128-bit counts, entry by entry: two hubs of 2^15 leaves (shared
    # in part, the leaves linked into a path) carry counts above 2^64 from level
    # 7 on and 128-bit bounds from level 6; 48 rows of 150 neighbours hold both
    # hubs last, so their neighbour-sum bounds reach 2^64 only in their third
    # 64-neighbour chunk (the 64-bit gather pass stops there and the row is
    # redone in 128 bits). Every level, t, t_j and 2000 samples, with grouped
    # rows and with one row per wave; with the width test before the combine
    # (automatic: level 7, where the leaves' level-6 sums are 128-bit; forced at
    # every level) and inside it, which covers both 128-bit-input routes of
    # vertices with high words in their top-level sums only.
    S = scc()
    g = gg.two_hubs()
    k = 8
    colors = gg.colors(g.n, k, seed=77)
    ot = O.Table(g, colors, k)
    print("two hubs: oracle table built", flush=True)
    ov, op = ot.sample(2000, seed=3)
    print("two hubs: oracle samples drawn", flush=True)
    dg = S.DeviceGraph.from_graph(g)
    for mode, width in GATHER_WIDTH:
        gt = S.Table(dg, colors, k, gather_mode=mode, width_test=width)
        info = gt.info()
        print(f"two hubs: modes {mode}, {width} 128-bit-input routes per level "
              f"{[list(info.wide_input_rows[h]) for h in range(k + 1)]}, per-lane width test "
              f"{info.lane_width_test:#x}, sorted sum rows {info.sorted_sum_rows:#x}", flush=True)
        if mode == S.GATHER_ROW:
            assert info.sorted_sum_rows >> 6 & 1, info.sorted_sum_rows
        if width == 2:
            assert info.lane_width_test == 0 and info.wide_input_rows[7][0] > 0, mode
        else:
            assert info.lane_width_test >> 7 & 1 and info.wide_input_rows[7][1] > 0, (mode, width)
        for h in (6, 7, 8):
            assert info.wide_vertices[h] > 0, (mode, h, list(info.wide_vertices))
        assert gt.totals()[0] >= 1 << 64
        assert_tables_equal(gt, ot, k, f"two hubs modes {mode}, {width}")
        gv, gp = gt.sample(2000, seed=3)
        assert np.array_equal(gv.cpu().numpy(), ov) and np.array_equal(gp.cpu().numpy(), op), (mode, width)
        print(f"two hubs: modes {mode}, {width} equal", flush=True)


@pytest.mark.parametrize("k,n,m", [(5, 3000, 12000), (8, 600, 1500)])
def test_combine_bytes_match_their_definition(k, n, m):
    # scc_combine_bytes against its definition from the exported records: at
    # level h, every vertex that has level h reads its own records of levels
    # 2..h-1 (10 B an entry), its dense neighbour sums of levels 1..h-1 (8 B an
    # entry; widths r_h'' binom(k-1, h'')), and writes its level-h record; level
    # k at colour-0 vertices only; the totals read level k and write 32 B a vertex
    from math import comb
    S = scc()
    g = gg.erdos_renyi(n, m, seed=71)
    colors = gg.colors(g.n, k, seed=72)
    gt = S.Table(S.DeviceGraph.from_graph(g), colors, k)
    assert all(gt.info().wide_vertices[h] == 0 for h in range(9))
    lens = {}
    for h in range(2, k + 1):
        off = gt.export_level(h)[0]
        lens[h] = np.diff(off).astype(np.int64)
    ws = {hs: O.num_shapes(hs) * comb(k - 1, hs) for hs in range(1, k)}
    zero = colors == 0
    cb, tb = gt.combine_bytes()
    for h in range(2, k + 1):
        per_v = 10 * lens[h] + sum(10 * lens[q] for q in range(2, h)) + sum(8 * ws[q] for q in range(1, h))
        want = int(per_v[zero].sum()) if h == k else int(per_v.sum())
        assert cb[h] == want, h
    assert tb == int(10 * lens[k].sum() + 32 * g.n)
