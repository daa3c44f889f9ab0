"""Biased colourings (Sec. 3.5) on the GPU vs the oracle, bit for bit.

* scc_color_biased equals the oracle's colouring for every k in [2, 8], several
  lambda (including the extremes 1/(k-1) and 2^-32) and ragged sizes.
* scc_colour_set_probability equals the oracle's probability (and j!/k^j for
  uniform colours).
* Tables and sample streams built on biased colourings equal the oracle's on
  random graphs for k = 4..8, under zero-rooting and round skipping.
* At the mid-size workload (Chung-Lu n = 1e6, m = 1e7, k = 6) with lambda =
  0.02: the k-star total equals sum_v prod_{j != c_v} n_j(v) (a closed form
  that holds for any colouring) and the table stores far fewer counts than
  under uniform colours.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import graphgen as gg
import oracle as O
from gpu_util import assert_tables_equal, random_graphs, scc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7, 8])
def test_biased_colours_equal_oracle(k):
    S = scc()
    for lam in (0.001, 0.05, 1.0 / (k - 1) if k > 1 else 0.5, 2.0 ** -32):
        L = min(O.lambda_units(lam), 2 ** 32 - 1)
        if (k - 1) * L > 2 ** 32:
            L -= 1
        lam = L / 2 ** 32
        for n in (1, 1000, 1_000_003):
            got = S.color_biased(n, k, lam, seed=5 + k, stream_id=n).cpu().numpy()
            ref = O.color_biased(n, k, L, seed=5 + k, stream=n)
            assert np.array_equal(got, ref), (k, lam, n)


def test_probabilities_equal_oracle():
    S = scc()
    for k in range(2, 9):
        for lam in (0.01, 0.1):
            L = O.lambda_units(lam)
            for j in range(1, k + 1):
                for z in (False, True):
                    assert S.colour_set_probability(k, lam, j, z) == pytest.approx(O.colour_set_prob(k, L, j, z),
                                                                                     rel=1e-14)
        assert S.colorful_probability(k) == pytest.approx(math.factorial(k) / k ** k, rel=1e-14)
    S_ = scc()
    with pytest.raises(S_.SccError) as e:
        S_.color_biased(10, 4, 0.5, seed=1)   # 3 * 0.5 > 1
    assert e.value.status == S_.EINVAL


@pytest.mark.parametrize("k", [4, 5, 6, 7, 8])
@pytest.mark.parametrize("rooting", [O.ROOT_ZERO, O.ROOT_BALANCED])
def test_tables_and_samples_on_biased_colourings(k, rooting):
    S = scc()
    lam = 0.12
    for name, g in random_graphs(k):
        dcol = S.color_biased(g.n, k, lam, seed=k, stream_id=len(name))
        colors = dcol.cpu().numpy()
        gt = S.Table(S.DeviceGraph.from_graph(g), dcol, k, rooting=rooting, validate=True)
        ot = O.Table(g, colors, k, rooting)
        assert_tables_equal(gt, ot, k, f"{name} biased")
        if ot.totals()[0]:
            gv, gp = gt.sample(500, seed=3, stream_id=1)
            ov, op = ot.sample(500, seed=3, stream=1)
            assert np.array_equal(gv.cpu().numpy(), ov) and np.array_equal(gp.cpu().numpy(), op), name


@pytest.mark.timeout(600)
def test_mid_workload_biased():
    S = scc()
    k = 6
    g = gg.chung_lu(1_000_000, 10_000_000, 2.1, 5e4, seed=2)
    dg = S.DeviceGraph.from_graph(g)
    dcol = S.color_biased(g.n, k, 0.02, seed=12)
    colors = dcol.cpu().numpy()
    bt = S.Table(dg, dcol, k)
    ut = S.Table(dg, gg.colors(g.n, k, seed=12), k)
    # far fewer colourful treelets: far fewer stored counts (the dense
    # neighbour-sum arrays keep their size)
    bi, ui = bt.info(), ut.info()
    assert sum(bi.nnz[h] for h in range(2, k + 1)) < sum(ui.nnz[h] for h in range(2, k + 1)) / 2
    assert bi.bytes < ui.bytes
    deg = np.diff(g.row_ptr)
    rows = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    nc = np.bincount(rows * k + colors[g.col_idx].astype(np.int64), minlength=g.n * k).reshape(g.n, k)
    prod = np.ones(g.n, dtype=object)
    for j in range(k):
        col = nc[:, j].astype(object)
        col[colors == j] = 1
        prod *= col
    star = next(r for r in range(O.num_shapes(k)) if O.shape_string(k, r) == "10" * (k - 1))
    assert bt.totals()[1][O.shape_unrooted(k, star)] == int(sum(prod))
