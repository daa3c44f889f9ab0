"""GPU sampler, classifier, catalog and AGS vs the oracle (bit-exact samples and classes).

The sampler's stream is fixed by (seed, stream id, sample index), so the GPU
samples must equal the oracle's vertex for vertex and parent for parent.
"""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from gpu_util import assert_samples_equal, build_pair, random_graphs, scc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("rooting", [O.ROOT_ZERO, O.ROOT_ALL])
@pytest.mark.parametrize("hub_degree", [0, 5])
def test_uniform_samples_equal(k, rooting, hub_degree):
    # hub_degree = 5: rows of degree > 5 draw neighbours from per-hub running sums
    for name, g in random_graphs(k):
        colors = gg.colors(g.n, k, seed=5 * k + rooting)
        gt, ot = build_pair(g, colors, k, rooting=rooting, hub_degree=hub_degree)
        if ot.totals()[0] == 0:
            continue
        assert_samples_equal(gt, ot, 300, seed=1000 + k, stream=rooting, label=name)


@pytest.mark.parametrize("k", [4, 5, 6, 7, 8])
@pytest.mark.parametrize("hub_degree", [0, 12])
def test_shape_restricted_samples_equal(k, hub_degree):
    g = gg.chung_lu(600, 2400, 2.2, 60, seed=50 + k)
    colors = gg.colors(g.n, k, seed=60 + k)
    gt, ot = build_pair(g, colors, k, hub_degree=hub_degree)
    t, tj = ot.totals()
    assert gt.totals() == (t, tj)
    for j, tot in enumerate(tj):
        if tot == 0:
            continue
        assert_samples_equal(gt, ot, 120, seed=7, stream=j, shape=j, label=f"k{k} shape {j}")


def test_sample_index_offsets_and_streams():
    g = gg.chung_lu(2000, 9000, 2.1, 300, seed=3)
    k = 6
    gt, ot = build_pair(g, gg.colors(g.n, k, seed=4), k)
    assert_samples_equal(gt, ot, 200, seed=99, stream=5, first=12345, label="offset")
    a, _ = gt.sample(64, seed=99, stream_id=5)
    b, _ = gt.sample(32, seed=99, stream_id=5, first_index=32)
    assert np.array_equal(a[32:].cpu().numpy(), b.cpu().numpy())


def test_samples_with_wide_counts():
    leaves = 1 << 16
    edges = [(0, i) for i in range(1, leaves + 1)] + [(i, i + 1) for i in range(1, 400)]
    g = gg.csr_from_edges(leaves + 1, np.array(edges, np.int64))
    colors = np.concatenate([[0], (np.arange(leaves) % 5) + 1]).astype(np.uint8)
    gt, ot = build_pair(g, colors, 6)
    assert_samples_equal(gt, ot, 200, seed=3, label="wide star")


@pytest.mark.parametrize("k", [3, 4, 5, 6, 7, 8])
def test_classify_equal(k):
    g = gg.chung_lu(1500, 7000, 2.2, 120, seed=70 + k)
    colors = gg.colors(g.n, k, seed=80 + k)
    gt, ot = build_pair(g, colors, k)
    if ot.totals()[0] == 0:
        pytest.skip("no colourful treelet")
    n = 400 if k < 8 else 60
    gv = assert_samples_equal(gt, ot, n, seed=5, label=f"classify k{k}")
    import torch
    code, cls = gt.classify(torch.as_tensor(gv).cuda())
    ocode, ocls = O.classify(g, k, gv)
    assert np.array_equal(code.cpu().numpy().view(np.uint32), ocode)
    assert np.array_equal(cls.cpu().numpy(), ocls)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7])
def test_catalog_equal(k):
    S = scc()
    cat = S.catalog(k, with_sigma=True, with_sigma_ij=(k <= 6))
    assert np.array_equal(cat["codes"], O.catalog_codes(k))
    for i, c in enumerate(cat["codes"][:400]):
        assert cat["sigma"][i] == O.spanning_trees(int(c), k)
        if cat["sigma_ij"] is not None:
            assert np.array_equal(cat["sigma_ij"][i], O.spanning_trees_by_shape(int(c), k))


@pytest.mark.timeout(300)
@pytest.mark.parametrize("k", [7, 8])
def test_catalog_sigma_ij_large_k(k):
    # spanning trees by shape at k = 7, 8 (the tree-shape table and the threaded cache)
    S = scc()
    cat = S.catalog(k, with_sigma=True, with_sigma_ij=True)
    rng = np.random.default_rng(k)
    pick = rng.choice(len(cat["codes"]), 40, replace=False)
    for i in list(pick) + [len(cat["codes"]) - 1]:
        c = int(cat["codes"][i])
        assert np.array_equal(cat["sigma_ij"][i], O.spanning_trees_by_shape(c, k)), i
        assert cat["sigma_ij"][i].sum() == cat["sigma"][i]


@pytest.mark.timeout(300)
def test_catalog_k8_matches_paper_and_oracle():
    # Sec. 5.2: 11117 distinct 8-graphlets; codes equal the oracle's catalog
    S = scc()
    cat = S.catalog(8, with_sigma=True)
    assert len(cat["codes"]) == 11117
    assert np.array_equal(cat["codes"], O.catalog_codes(8))
    rng = np.random.default_rng(1)
    for i in rng.choice(11117, 50, replace=False):
        assert cat["sigma"][i] == O.spanning_trees(int(cat["codes"][i]), 8)


def test_ags_equal_on_star_plus_path():
    k = 4
    leaves, plen = 80, 9
    edges = [(0, i) for i in range(1, leaves + 1)] + [(leaves + 1 + i, leaves + 2 + i) for i in range(plen - 1)]
    g = gg.csr_from_edges(leaves + 1 + plen, np.array(edges, np.int64))
    colors = gg.colors(g.n, k, seed=3)
    gt, ot = build_pair(g, colors, k)
    r_gpu = gt.ags(cbar=100, round_size=50, budget=6000, seed=11, stream_id=2)
    r_orc = ot.ags(cbar=100, round_size=50, budget=6000, seed=11, stream=2)
    for key in ["hits", "w", "n_j", "round_shapes"]:
        assert np.array_equal(r_gpu[key], r_orc[key]), key


def test_ags_equal_on_chung_lu_k5():
    g = gg.chung_lu(3000, 12000, 2.2, 200, seed=31)
    k = 5
    gt, ot = build_pair(g, gg.colors(g.n, k, seed=32), k)
    r_gpu = gt.ags(cbar=50, round_size=500, budget=20000, seed=8, stream_id=1)
    r_orc = ot.ags(cbar=50, round_size=500, budget=20000, seed=8, stream=1)
    for key in ["hits", "w", "n_j", "round_shapes"]:
        assert np.array_equal(r_gpu[key], r_orc[key]), key


def test_ags_printed_rule_at_round_size_one():
    # rounds of one sample are the printed algorithm: the GPU controller makes
    # the oracle's choices draw by draw (the oracle is pinned to a transcription)
    g = gg.chung_lu(120, 300, 2.2, 25, seed=31)
    k = 5
    gt, ot = build_pair(g, gg.colors(g.n, k, seed=8), k)
    r_gpu = gt.ags(cbar=20, round_size=1, budget=2000, seed=8, stream_id=1)
    r_orc = ot.ags(cbar=20, round_size=1, budget=2000, seed=8, stream=1)
    assert len(set(r_orc["round_shapes"].tolist())) > 1
    for key in ["hits", "w", "n_j", "round_shapes"]:
        assert np.array_equal(r_gpu[key], r_orc[key]), key


def test_estimates_equal_oracle():
    # Sec. 2.2 estimators from the GPU's own samples and classes, and from AGS
    g = gg.chung_lu(3000, 12000, 2.2, 200, seed=31)
    k = 5
    gt, ot = build_pair(g, gg.colors(g.n, k, seed=32), k)
    v, _ = gt.sample(20000, seed=4)
    _, cls = gt.classify(v)
    hits = np.bincount(cls.cpu().numpy(), minlength=O.num_classes(k)).astype(np.int64)
    for pk in (0.0, 0.01):
        gc, gg_ = gt.estimate(hits, n=20000, p_k=pk)
        oc, og = O.estimate(ot, hits, n=20000, pk=pk)
        assert np.allclose(gc, oc, rtol=1e-14, atol=0) and np.allclose(gg_, og, rtol=1e-14, atol=0)
    r = gt.ags(cbar=50, round_size=500, budget=20000, seed=8, stream_id=1)
    gc, gg_ = gt.estimate(r["hits"], w=r["w"])
    oc, og = O.estimate(ot, r["hits"], w=r["w"])
    assert np.array_equal(gc, oc) and np.allclose(gg_, og, rtol=1e-14, atol=0)
    assert (gc > 0).sum() == (r["hits"] > 0).sum()
